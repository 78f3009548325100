"""MI355X (gfx950) KmerCo: countBF insertion and threshold classification.

The compute lives in ``libkmerco_hip.so`` (hand-written HIP kernels behind the
C ABI of ``include/kmerco.h``); this package is its Python binding.
"""
from .kmerco import (  # noqa: F401
    KC_EDEVICE,
    KC_EINVAL,
    KC_ENOMEM,
    KC_ERANGE,
    KC_ESTATE,
    KC_OK,
    Batch,
    CountBF,
    KmercoError,
    LIB_PATH,
    SIGNATURES,
    Server,
    dims,
    eta,
    filter_bytes,
    key_words,
    load_library,
    pack_read_sets,
    parse_fastx,
    read_fastx,
    run_kmerco,
    scratch_bytes,
    strerror,
)
