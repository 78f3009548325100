"""ctypes binding of the gfx950 KmerCo library (``include/kmerco.h``).

Argument marshalling only: torch tensors supply device memory and streams;
every step of the insertion and classification phases runs in the library's
HIP kernels.  The library must be built (``paper_2305_07545_amd.build``); there
is no fallback path.

64-bit keys, words and offsets travel as ``torch.int64`` tensors holding the
unsigned bit patterns.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmerco_hip.so")

KC_OK, KC_EINVAL, KC_ENOMEM, KC_ERANGE, KC_EDEVICE, KC_ESTATE = 0, -1, -2, -3, -4, -5


class KmercoError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class kc_layout(ctypes.Structure):
    _fields_ = [("X", ctypes.c_uint64), ("Y", ctypes.c_uint64),
                ("alpha", ctypes.c_uint32), ("k_h", ctypes.c_uint32)]


class kc_set(ctypes.Structure):
    _fields_ = [("filter", ctypes.c_void_p),
                ("first_base", ctypes.c_uint64), ("n_bases", ctypes.c_uint64),
                ("k", ctypes.c_uint32), ("tau", ctypes.c_uint32),
                ("distinct_dev", ctypes.c_void_p), ("distinct_cap", ctypes.c_uint64),
                ("n_distinct_dev", ctypes.c_void_p), ("n_windows_dev", ctypes.c_void_p),
                ("trust_dev", ctypes.c_void_p), ("n_trust_dev", ctypes.c_void_p),
                ("err_dev", ctypes.c_void_p), ("n_err_dev", ctypes.c_void_p),
                ("class_cap", ctypes.c_uint64)]


KC_BATCH_RESET, KC_BATCH_GRAPH, KC_BATCH_TUNE = 1, 2, 4
SET_ALIGN = 4096


class kc_plan(ctypes.Structure):
    _fields_ = [("path", ctypes.c_uint32), ("region_cells", ctypes.c_uint32),
                ("n_regions", ctypes.c_uint32), ("n_parts", ctypes.c_uint32),
                ("chunk", ctypes.c_uint64), ("n_chunks", ctypes.c_uint64),
                ("carried", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


PATH_NAMES = {0: "direct", 1: "binned", 2: "partitioned"}


class kc_server_config(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("lane_bases", ctypes.c_uint64),
                ("lane_reads", ctypes.c_uint64), ("lane_requests", ctypes.c_uint32),
                ("lanes", ctypes.c_uint32)]


class kc_request(ctypes.Structure):
    _fields_ = [("session", ctypes.c_uint32), ("op", ctypes.c_uint32),
                ("tau", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("reads_host", ctypes.c_void_p), ("offsets_host", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint64), ("trust_dev", ctypes.c_void_p),
                ("err_dev", ctypes.c_void_p), ("class_cap", ctypes.c_uint64)]


class kc_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("done", ctypes.c_uint32),
                ("n_windows", ctypes.c_uint64), ("distinct_first", ctypes.c_uint64),
                ("n_new", ctypes.c_uint64), ("n_trust", ctypes.c_uint64),
                ("n_err", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_issue", ctypes.c_double), ("t_done", ctypes.c_double)]


class kc_server_stats(ctypes.Structure):
    _fields_ = [("session_bytes", ctypes.c_uint64), ("staging_bytes", ctypes.c_uint64),
                ("sessions_open", ctypes.c_uint32), ("sessions_waiting", ctypes.c_uint32),
                ("requests_done", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("batched_requests", ctypes.c_uint64), ("plain_requests", ctypes.c_uint64),
                ("max_batch", ctypes.c_uint32), ("lanes_in_flight_max", ctypes.c_uint32)]


KC_OP_INSERT, KC_OP_CLASSIFY = 1, 2

_lib = None

# every symbol include/kmerco.h declares, with (restype, argtypes)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_i = ctypes.c_int
SIGNATURES = {
    "kc_strerror": (ctypes.c_char_p, [_i]),
    "kc_version": (_i, []),
    "kc_dims": (_i, [ctypes.c_double, ctypes.c_double, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "kc_parse_fastx": (_i, [_vp, _u64, _u32, _vp, _u64, _vp, _u64, ctypes.POINTER(_u64),
                            ctypes.POINTER(_u64)]),
    "kc_eta": (_u32, [_u32]),
    "kc_filter_bytes": (_u64, [ctypes.POINTER(kc_layout)]),
    "kc_scratch_bytes": (_u64, [ctypes.POINTER(kc_layout), _u64]),
    "kc_create": (_i, [ctypes.POINTER(kc_layout), _vp, _i, _vp, ctypes.POINTER(_vp)]),
    "kc_create_in": (_i, [ctypes.POINTER(kc_layout), _vp, _i, _u32, _vp, _u64, _u64, _vp,
                          ctypes.POINTER(_vp)]),
    "kc_destroy": (None, [_vp]),
    "kc_reserve": (_i, [_vp, _u64]),
    "kc_insert": (_i, [_vp, _vp, _vp, _u64, _u64, _u32, _vp, _u64, _vp, _vp, _vp]),
    "kc_classify": (_i, [_vp, _vp, _vp, _u64, _u32, _vp, _vp, _vp, _vp, _vp]),
    "kc_insert_classify": (_i, [_vp, _vp, _vp, _u64, _u64, _u32, _u32, _vp, _u64, _vp, _vp,
                                _vp, _vp, _vp, _vp, _u64, _vp]),
    "kc_insert_classify_noalloc": (_i, [_vp, _vp, _vp, _u64, _u64, _u32, _u32, _vp, _u64, _vp,
                                        _vp, _vp, _vp, _vp, _vp, _u64, _vp]),
    "kc_query": (_i, [_vp, _vp, _u64, _vp, _vp]),
    "kc_sync": (_i, [_vp]),
    "kc_get_layout": (_i, [_vp, ctypes.POINTER(kc_layout)]),
    "kc_get_plan": (_i, [_vp, _u64, ctypes.POINTER(kc_plan)]),
    "kc_reset": (_i, [_vp, _vp]),
    "kc_profile": (_i, [_vp, _i]),
    "kc_profile_phases": (_i, [_vp, _u32]),
    "kc_profile_read": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_u64), _u32]),
    "kc_phase_name": (ctypes.c_char_p, [_u32]),
    "kc_batch_create": (_i, [ctypes.POINTER(_vp)]),
    "kc_batch_destroy": (None, [_vp]),
    "kc_batch_insert": (_i, [_vp, ctypes.POINTER(kc_set), _u32, _vp, _vp, _u64, _u64, _u32, _vp]),
    "kc_batch_get_tile": (_i, [_vp, ctypes.POINTER(_u64)]),
    "kc_batch_set_tile": (_i, [_vp, _u64]),
    "kc_batch_profile": (_i, [_vp, _i]),
    "kc_batch_profile_read": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_u64), _u32]),
    "kc_batch_sync": (_i, [_vp]),
    "kc_server_create": (_i, [ctypes.POINTER(kc_server_config), ctypes.POINTER(_vp)]),
    "kc_server_destroy": (None, [_vp]),
    "kc_server_open": (_i, [_vp, ctypes.POINTER(kc_layout), _u32, _u64, ctypes.POINTER(_u32)]),
    "kc_server_close": (_i, [_vp, _u32]),
    "kc_server_submit": (_i, [_vp, ctypes.POINTER(kc_request), ctypes.POINTER(_u64)]),
    "kc_server_pump": (_i, [_vp, ctypes.POINTER(_u32)]),
    "kc_server_wait": (_i, [_vp, _u64]),
    "kc_server_result": (_i, [_vp, _u64, ctypes.POINTER(kc_result)]),
    "kc_server_release": (_i, [_vp, _u64]),
    "kc_server_read_distinct": (_i, [_vp, _u32, _u64, _u64, _vp]),
    "kc_server_read_words": (_i, [_vp, _u32, _vp]),
    "kc_server_stats_get": (_i, [_vp, ctypes.POINTER(kc_server_stats)]),
    "kc_server_now": (ctypes.c_double, [_vp]),
}

PHASES = ["ingest", "claim", "increment", "claim_increment", "resolve", "scan", "scatter",
          "classify_mark", "classify_scatter", "query", "reset", "bin_count", "bin_bucket",
          "region", "tile_count", "bin_region", "bin_part", "part_count", "valid_windows",
          "winners"]


def load_library():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"KmerCo HIP library not built ({LIB_PATH}); "
                               "run paper_2305_07545_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load_library().kc_strerror(status).decode()


def _check(status: int, what: str):
    if status != KC_OK:
        raise KmercoError(status, what)


def dims(n_items: float, fpp: float = 0.001):
    """Eq. (1) countBF dimensions (X, Y)."""
    X = ctypes.c_uint64(0)
    Y = ctypes.c_uint64(0)
    _check(load_library().kc_dims(float(n_items), float(fpp), ctypes.byref(X), ctypes.byref(Y)),
           "kc_dims")
    return int(X.value), int(Y.value)


KC_FASTX_ONE_SEQUENCE = 1


def key_words(k) -> int:
    """uint64 words per k-mer key: 1 for k <= 32, 2 (low, high) for 33..64."""
    return 2 if k is not None and k > 32 else 1


def parse_fastx(data, one_sequence: bool = False):
    """FASTA or FASTQ text (bytes-like or a uint8 numpy array, host memory)
    -> (reads uint8, offsets uint64) for the insert calls, by
    kc_parse_fastx: one read per record, or one read for the whole text
    with ``one_sequence``."""
    import numpy as np
    lib = load_library()
    buf = data if isinstance(data, np.ndarray) else np.frombuffer(data, dtype=np.uint8)
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    flags = KC_FASTX_ONE_SEQUENCE if one_sequence else 0
    nb, nr = ctypes.c_uint64(0), ctypes.c_uint64(0)
    text = buf.ctypes.data if buf.size else None
    st = lib.kc_parse_fastx(text, buf.size, flags, None, 0, None, 0, ctypes.byref(nb),
                            ctypes.byref(nr))
    if st not in (KC_OK, KC_ERANGE):
        _check(st, "kc_parse_fastx")
    seq = np.empty(nb.value, dtype=np.uint8)
    offs = np.empty(nr.value + 1, dtype=np.uint64)
    _check(lib.kc_parse_fastx(text, buf.size, flags, seq.ctypes.data if seq.size else None,
                              seq.size, offs.ctypes.data, offs.size, ctypes.byref(nb),
                              ctypes.byref(nr)), "kc_parse_fastx")
    return seq, offs


def read_fastx(path: str, one_sequence: bool = False):
    """parse_fastx of a file, memory-mapped."""
    import mmap

    import numpy as np
    with open(path, "rb") as f:
        if os.fstat(f.fileno()).st_size == 0:
            return parse_fastx(b"", one_sequence)
        with mmap.mmap(f.fileno(), 0, access=mmap.ACCESS_READ) as m:
            return parse_fastx(np.frombuffer(m, dtype=np.uint8), one_sequence)


def eta(alpha: int) -> int:
    return int(load_library().kc_eta(alpha))


def filter_bytes(X: int, Y: int, alpha: int = 8, k_h: int = 1) -> int:
    """Bytes of the countBF words of a layout (0 if invalid)."""
    L = kc_layout(X, Y, alpha, k_h)
    return int(load_library().kc_filter_bytes(ctypes.byref(L)))


def scratch_bytes(X: int, Y: int, max_bases: int, alpha: int = 8, k_h: int = 1) -> int:
    """Device bytes a handle of this layout allocates for inserts of up to
    max_bases bases (what CountBF.reserve(max_bases) allocates; 0 if the
    layout is invalid).  Host only."""
    L = kc_layout(X, Y, alpha, k_h)
    return int(load_library().kc_scratch_bytes(ctypes.byref(L), int(max_bases)))


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class CountBF:
    """A countBF resident in device memory, driven by the HIP library.

    ``words`` (int64[X*Y]) is allocated here unless given; with ``zero=True``
    the library clears it and the filter starts empty.  ``k``: the k-mer
    length the given words already hold (a resumed countBF).  ``scratch``: a
    device uint8 tensor of at least ``scratch_bytes(X, Y, max_bases, ...)``
    bytes that holds every buffer of the handle (kc_create_in): no call then
    allocates device memory, and inserts of more than ``max_bases`` bases
    fail."""

    def __init__(self, X: int, Y: int, alpha: int = 8, k_h: int = 1, words=None,
                 zero: bool = True, device=None, stream=None, k: int = 0, scratch=None,
                 max_bases: int = 0):
        self.lib = load_library()
        self.layout = kc_layout(X, Y, alpha, k_h)
        dev = torch.device("cuda") if device is None else torch.device(device)
        if words is None:
            words = torch.empty(X * Y, dtype=torch.int64, device=dev)
        _require(words, torch.int64, "words")
        if words.numel() != X * Y:
            raise ValueError("words must hold X*Y cells")
        self.words = words
        self.device = words.device
        if scratch is not None:
            _require(scratch, torch.uint8, "scratch")
            if scratch.device != self.device:
                raise ValueError("scratch must be on the words' device")
        self.scratch = scratch  # kept alive as long as the handle
        h = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(self.lib.kc_create_in(
                ctypes.byref(self.layout), _ptr(words), int(zero), int(k), _ptr(scratch),
                0 if scratch is None else scratch.numel(), int(max_bases), _stream_ptr(stream),
                ctypes.byref(h)), "kc_create_in")
        self._h = h
        self.k = k or None  # k of the inserts (keys of k > 32 bases take two words)
        self.n_distinct = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.n_windows = torch.zeros(1, dtype=torch.int64, device=self.device)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.kc_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def reserve(self, max_bases: int):
        with torch.cuda.device(self.device):
            _check(self.lib.kc_reserve(self._h, int(max_bases)), "kc_reserve")

    def insert(self, reads, offsets, k: int, distinct=None, distinct_cap=None,
               n_distinct=None, n_windows=None, stream=None):
        """Insertion phase over one read batch (async).  Appends this call's
        distinct keys to ``distinct`` at ``n_distinct`` (device counters)."""
        _require(reads, torch.uint8, "reads")
        _require(offsets, torch.int64, "offsets")
        n_reads = offsets.numel() - 1
        n_bases = reads.numel()
        if n_reads < 0:
            raise ValueError("offsets needs n_reads + 1 entries")
        w = key_words(k)
        if distinct is None:
            distinct = torch.empty(max(1, n_bases) * w, dtype=torch.int64, device=self.device)
        _require(distinct, torch.int64, "distinct")
        cap = distinct.numel() // w if distinct_cap is None else int(distinct_cap)
        n_distinct = self.n_distinct if n_distinct is None else n_distinct
        n_windows = self.n_windows if n_windows is None else n_windows
        with torch.cuda.device(self.device):
            _check(self.lib.kc_insert(self._h, _ptr(reads), _ptr(offsets), n_reads, n_bases, k,
                                      _ptr(distinct), cap, _ptr(n_distinct), _ptr(n_windows),
                                      _stream_ptr(stream)), "kc_insert")
        self.k = k
        return distinct

    def insert_classify(self, reads, offsets, k: int, tau: int, distinct=None, trust=None,
                        err=None, n_distinct=None, n_windows=None, n_trust=None, n_err=None,
                        class_cap=None, stream=None):
        """Both phases for one read batch (async): insertion, then the split
        of this call's distinct keys at tau.  Returns (distinct, trust,
        n_trust, err, n_err)."""
        _require(reads, torch.uint8, "reads")
        _require(offsets, torch.int64, "offsets")
        n_reads = offsets.numel() - 1
        n_bases = reads.numel()
        if n_reads < 0:
            raise ValueError("offsets needs n_reads + 1 entries")
        w = key_words(k)
        room = max(1, n_bases) * w
        if distinct is None:
            distinct = torch.empty(room, dtype=torch.int64, device=self.device)
        if trust is None:
            trust = torch.empty(room, dtype=torch.int64, device=self.device)
        if err is None:
            err = torch.empty(room, dtype=torch.int64, device=self.device)
        for t, nm in ((distinct, "distinct"), (trust, "trust"), (err, "err")):
            _require(t, torch.int64, nm)
        cap_te = min(trust.numel(), err.numel()) // w if class_cap is None else int(class_cap)
        n_distinct = self.n_distinct if n_distinct is None else n_distinct
        n_windows = self.n_windows if n_windows is None else n_windows
        if n_trust is None:
            n_trust = torch.zeros(1, dtype=torch.int64, device=self.device)
        if n_err is None:
            n_err = torch.zeros(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self.lib.kc_insert_classify(
                self._h, _ptr(reads), _ptr(offsets), n_reads, n_bases, k, int(tau),
                _ptr(distinct), distinct.numel() // w, _ptr(n_distinct), _ptr(n_windows),
                _ptr(trust), _ptr(n_trust), _ptr(err), _ptr(n_err), cap_te,
                _stream_ptr(stream)), "kc_insert_classify")
        self.k = k
        return distinct, trust, n_trust, err, n_err

    def insert_classify_noalloc(self, reads, offsets, k: int, tau: int, distinct, trust, err,
                                n_distinct, n_windows, n_trust, n_err, stream=None):
        """insert_classify through kc_insert_classify_noalloc: the call's
        scratch is the library's fixed per-device array, nothing is
        allocated (every output buffer and counter must be given)."""
        for t, nm in ((distinct, "distinct"), (trust, "trust"), (err, "err"),
                      (n_distinct, "n_distinct"), (n_windows, "n_windows"),
                      (n_trust, "n_trust"), (n_err, "n_err")):
            _require(t, torch.int64, nm)
        _require(reads, torch.uint8, "reads")
        _require(offsets, torch.int64, "offsets")
        w = key_words(k)
        with torch.cuda.device(self.device):
            _check(self.lib.kc_insert_classify_noalloc(
                self._h, _ptr(reads), _ptr(offsets), offsets.numel() - 1, reads.numel(), k,
                int(tau), _ptr(distinct), distinct.numel() // w, _ptr(n_distinct),
                _ptr(n_windows), _ptr(trust), _ptr(n_trust), _ptr(err), _ptr(n_err),
                min(trust.numel(), err.numel()) // w, _stream_ptr(stream)),
                "kc_insert_classify_noalloc")
        self.k = k

    def classify(self, keys, n_keys, tau: int, trust=None, err=None, n_trust=None, n_err=None,
                 keys_cap=None, stream=None):
        """Classification phase (async); returns (trust, n_trust, err, n_err)
        device tensors."""
        _require(keys, torch.int64, "keys")
        w = key_words(self.k)
        cap = keys.numel() // w if keys_cap is None else int(keys_cap)
        if trust is None:
            trust = torch.empty(max(1, cap) * w, dtype=torch.int64, device=self.device)
        if err is None:
            err = torch.empty(max(1, cap) * w, dtype=torch.int64, device=self.device)
        if n_trust is None:
            n_trust = torch.zeros(1, dtype=torch.int64, device=self.device)
        if n_err is None:
            n_err = torch.zeros(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self.lib.kc_classify(self._h, _ptr(keys), _ptr(n_keys), cap, int(tau),
                                        _ptr(trust), _ptr(n_trust), _ptr(err), _ptr(n_err),
                                        _stream_ptr(stream)), "kc_classify")
        return trust, n_trust, err, n_err

    def query(self, keys, freq=None, stream=None):
        _require(keys, torch.int64, "keys")
        n = keys.numel() // key_words(self.k)
        if freq is None:
            freq = torch.empty(max(1, n), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(self.lib.kc_query(self._h, _ptr(keys), n, _ptr(freq), _stream_ptr(stream)),
                   "kc_query")
        return freq[:n]

    def plan(self, n_bases: int) -> dict:
        """kc_get_plan: path, region size, regions, partitions and chunking
        of an insert of n_bases bases."""
        p = kc_plan()
        _check(self.lib.kc_get_plan(self._h, int(n_bases), ctypes.byref(p)), "kc_get_plan")
        d = {f: getattr(p, f) for f, _ in kc_plan._fields_}
        d["path"] = PATH_NAMES.get(d["path"], str(d["path"]))
        return d

    def reset(self, stream=None):
        """Clear the countBF (async): empty filter, k unset."""
        with torch.cuda.device(self.device):
            _check(self.lib.kc_reset(self._h, _stream_ptr(stream)), "kc_reset")
        self.k = None

    def profile(self, enable: bool = True, phases=None):
        """Time every phase (or only the named ones) of the following calls."""
        if phases is None:
            _check(self.lib.kc_profile(self._h, int(enable)), "kc_profile")
        else:
            mask = 0
            for ph in phases:
                mask |= 1 << PHASES.index(ph)
            _check(self.lib.kc_profile_phases(self._h, mask if enable else 0),
                   "kc_profile_phases")

    def profile_read(self):
        """{phase: (total ms, launches)} of the kernels recorded since the
        last read (waits for them)."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_uint64 * n)()
        with torch.cuda.device(self.device):
            _check(self.lib.kc_profile_read(self._h, ms, cnt, n), "kc_profile_read")
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    def sync(self):
        """Wait for the filter's work; raises on a sticky device error."""
        with torch.cuda.device(self.device):
            _check(self.lib.kc_sync(self._h), "kc_sync")

    def save(self, path, distinct=None, n_distinct=None):
        """Checkpoint the countBF (its words, layout and k) to an ``.npz``
        file, with the distinct list so far when ``distinct`` is given (its
        first ``n_distinct`` keys; the filter's own count by default).  The
        file holds plain arrays only (no pickles).  Synchronous."""
        import numpy as np
        self.sync()
        layout = np.array([self.layout.X, self.layout.Y, self.layout.alpha, self.layout.k_h,
                           0 if self.k is None else self.k], dtype=np.uint64)
        arrays = {"layout": layout, "words": self.words.cpu().numpy().view(np.uint64)}
        if distinct is not None:
            n = int((self.n_distinct if n_distinct is None else n_distinct).item())
            w = key_words(self.k)
            arrays["distinct"] = distinct[:n * w].cpu().numpy().view(np.uint64)
        with open(path, "wb") as fh:
            np.savez(fh, **arrays)

    @classmethod
    def load(cls, path, device=None, stream=None):
        """A countBF resumed from a ``save`` checkpoint: later inserts continue
        it as if the saved inserts and they had been one call.  Returns
        (countbf, distinct), distinct being the saved list as a device
        tensor (None when none was saved); the filter's n_distinct starts at
        its length."""
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            X, Y, alpha, k_h, k = (int(v) for v in z["layout"])
            words = torch.from_numpy(z["words"].view(np.int64).copy())
            distinct = z["distinct"].view(np.int64).copy() if "distinct" in z.files else None
        dev = torch.device("cuda") if device is None else torch.device(device)
        # the handle itself resumes with k: classify and query read keys of
        # its width, and inserts of another k are refused
        bf = cls(X, Y, alpha, k_h, words=words.to(dev), zero=False, device=dev, stream=stream, k=k)
        if distinct is not None:
            distinct = torch.from_numpy(distinct).to(dev)
            bf.n_distinct.fill_(distinct.numel() // key_words(bf.k))
        return bf, distinct


def run_kmerco(reads, offsets, k: int, tau: int, X: int, Y: int, alpha: int = 8, k_h: int = 1,
               stream=None, fused: bool = True):
    """Both phases on a fresh countBF.  Returns host numpy arrays
    (words, distinct, trust, err, n_windows) as uint64.  fused: one
    kc_insert_classify call; else kc_insert then kc_classify."""
    bf = CountBF(X, Y, alpha, k_h, stream=stream)
    if fused:
        distinct, trust, n_trust, err, n_err = bf.insert_classify(reads, offsets, k, tau,
                                                                  stream=stream)
    else:
        distinct = bf.insert(reads, offsets, k, stream=stream)
        trust, n_trust, err, n_err = bf.classify(distinct, bf.n_distinct, tau, stream=stream)
    bf.sync()
    nd = int(bf.n_distinct.item())
    nt = int(n_trust.item())
    ne = int(n_err.item())
    w = key_words(k)
    u = lambda t: t.cpu().numpy().view("uint64")  # noqa: E731
    lst = lambda t, n: u(t[:n * w]).reshape(-1, 2) if w == 2 else u(t[:n])  # noqa: E731
    out = (u(bf.words), lst(distinct, nd), lst(trust, nt), lst(err, ne),
           int(bf.n_windows.item()))
    bf.close()
    return out


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

def pack_read_sets(sets):
    """Concatenate read sets [(reads uint8, offsets uint64), ...] into one
    buffer in which every set starts at a multiple of SET_ALIGN bases; the
    gaps are filled with one read of 'N' bases (no valid k-mer).  Returns
    (reads, offsets, [(first_base, n_bases, first_read, n_reads)])."""
    import numpy as np
    parts, offs, spans = [], [np.zeros(1, dtype=np.uint64)], []
    pos = 0
    n_reads = 0
    for reads, offsets in sets:
        reads = np.asarray(reads, dtype=np.uint8)
        offsets = np.asarray(offsets, dtype=np.uint64)
        pad = (-pos) % SET_ALIGN
        if pad:
            parts.append(np.full(pad, ord("N"), dtype=np.uint8))
            offs.append(np.array([pos + pad], dtype=np.uint64))
            pos += pad
            n_reads += 1
        nb = int(offsets[-1])
        nr = len(offsets) - 1
        spans.append((pos, nb, n_reads, nr))
        parts.append(reads[:nb])
        if nr:
            offs.append(offsets[1:] + np.uint64(pos))
        pos += nb
        n_reads += nr
    reads = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
    return reads, np.concatenate(offs).astype(np.uint64), spans


class Batch:
    """kc_batch: insert many read sets, each into its own CountBF, with one
    launch per phase."""

    def __init__(self):
        self.lib = load_library()
        h = ctypes.c_void_p(None)
        _check(self.lib.kc_batch_create(ctypes.byref(h)), "kc_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.kc_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    @property
    def tile(self) -> int:
        t = ctypes.c_uint64(0)
        _check(self.lib.kc_batch_get_tile(self._h, ctypes.byref(t)), "kc_batch_get_tile")
        return int(t.value)

    @tile.setter
    def tile(self, value: int):
        _check(self.lib.kc_batch_set_tile(self._h, int(value)), "kc_batch_set_tile")

    def insert(self, entries, reads, offsets, reset=False, graph=False, tune=False, stream=None):
        """entries: list of dicts with keys filter (CountBF), first_base,
        n_bases, k, tau, distinct, n_distinct, n_windows, and optionally
        trust, n_trust, err, n_err (device tensors)."""
        _require(reads, torch.uint8, "reads")
        _require(offsets, torch.int64, "offsets")
        arr = (kc_set * len(entries))()
        for i, e in enumerate(entries):
            q = arr[i]
            q.filter = e["filter"].handle
            q.first_base = int(e["first_base"])
            q.n_bases = int(e["n_bases"])
            q.k = int(e["k"])
            q.tau = int(e.get("tau", 0))
            q.distinct_dev = e["distinct"].data_ptr()
            q.distinct_cap = int(e.get("distinct_cap", e["distinct"].numel()))
            q.n_distinct_dev = e["n_distinct"].data_ptr()
            q.n_windows_dev = e["n_windows"].data_ptr() if e.get("n_windows") is not None else None
            if e.get("trust") is not None:
                q.trust_dev = e["trust"].data_ptr()
                q.n_trust_dev = e["n_trust"].data_ptr()
                q.err_dev = e["err"].data_ptr()
                q.n_err_dev = e["n_err"].data_ptr()
                q.class_cap = int(e.get("class_cap", min(e["trust"].numel(), e["err"].numel())))
        flags = (KC_BATCH_RESET if reset else 0) | (KC_BATCH_GRAPH if graph else 0) | \
                (KC_BATCH_TUNE if tune else 0)
        with torch.cuda.device(reads.device):
            _check(self.lib.kc_batch_insert(self._h, arr, len(entries), _ptr(reads), _ptr(offsets),
                                            offsets.numel() - 1, reads.numel(), flags,
                                            _stream_ptr(stream)), "kc_batch_insert")

    def profile(self, enable: bool = True):
        _check(self.lib.kc_batch_profile(self._h, int(enable)), "kc_batch_profile")

    def profile_read(self):
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_uint64 * n)()
        _check(self.lib.kc_batch_profile_read(self._h, ms, cnt, n), "kc_batch_profile_read")
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    def sync(self):
        _check(self.lib.kc_batch_sync(self._h), "kc_batch_sync")


def _host_ptr(a):
    """Address of a host buffer: a numpy array or a CPU torch tensor."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda or not a.is_contiguous():
            raise ValueError("request buffers must be contiguous host memory")
        return a.data_ptr()
    import numpy as np
    if not isinstance(a, np.ndarray) or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("request buffers must be contiguous host memory")
    return a.ctypes.data


class Server:
    """kc_server: sessions of device-resident countBFs served by a request
    loop with continuous batching (see the kc_server entry points)."""

    def __init__(self, memory_budget: int, lane_bases: int, lane_reads: int,
                 lane_requests: int = 64, lanes: int = 2):
        self.lib = load_library()
        cfg = kc_server_config(int(memory_budget), int(lane_bases), int(lane_reads),
                               int(lane_requests), int(lanes))
        h = ctypes.c_void_p(None)
        _check(self.lib.kc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "kc_server_create")
        self._h = h
        self._keep = {}  # ticket -> host buffers the request reads from

    def close_server(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.kc_server_destroy(self._h)
            self._h = ctypes.c_void_p(None)
            self._keep.clear()

    def __del__(self):
        try:
            self.close_server()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def open(self, X: int, Y: int, k: int, distinct_cap: int, alpha: int = 8, k_h: int = 1) -> int:
        sid = ctypes.c_uint32(0)
        lay = kc_layout(int(X), int(Y), int(alpha), int(k_h))
        _check(self.lib.kc_server_open(self._h, ctypes.byref(lay), int(k), int(distinct_cap),
                                       ctypes.byref(sid)), "kc_server_open")
        return int(sid.value)

    def close(self, session: int):
        _check(self.lib.kc_server_close(self._h, int(session)), "kc_server_close")

    def submit(self, session: int, reads=None, offsets=None, classify: bool = False,
               insert: bool = True, tau: int = 0, trust=None, err=None) -> int:
        """reads: uint8 host buffer, offsets: uint64 host CSR (offsets[0] == 0);
        trust/err: device int64 tensors for a classify request."""
        q = kc_request()
        q.session = int(session)
        q.op = (KC_OP_INSERT if insert else 0) | (KC_OP_CLASSIFY if classify else 0)
        q.tau = int(tau)
        keep = []
        if insert:
            q.reads_host = _host_ptr(reads)
            q.offsets_host = _host_ptr(offsets)
            q.n_reads = (offsets.numel() if isinstance(offsets, torch.Tensor) else len(offsets)) - 1
            keep += [reads, offsets]
        if classify:
            _require(trust, torch.int64, "trust")
            _require(err, torch.int64, "err")
            q.trust_dev = trust.data_ptr()
            q.err_dev = err.data_ptr()
            q.class_cap = min(trust.numel(), err.numel())
            keep += [trust, err]
        t = ctypes.c_uint64(0)
        _check(self.lib.kc_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)),
               "kc_server_submit")
        self._keep[int(t.value)] = keep
        return int(t.value)

    def pump(self) -> int:
        n = ctypes.c_uint32(0)
        _check(self.lib.kc_server_pump(self._h, ctypes.byref(n)), "kc_server_pump")
        return int(n.value)

    def wait(self, ticket: int = 0):
        _check(self.lib.kc_server_wait(self._h, int(ticket)), "kc_server_wait")

    def result(self, ticket: int) -> dict:
        r = kc_result()
        _check(self.lib.kc_server_result(self._h, int(ticket), ctypes.byref(r)),
               "kc_server_result")
        if r.done:
            self._keep.pop(int(ticket), None)
        return {f: getattr(r, f) for f, _ in kc_result._fields_}

    def release(self, ticket: int):
        """Forget a done request's result (kc_server_release)."""
        _check(self.lib.kc_server_release(self._h, int(ticket)), "kc_server_release")
        self._keep.pop(int(ticket), None)

    def read_distinct(self, session: int, first: int, n: int):
        import numpy as np
        out = np.zeros(max(int(n), 1), dtype=np.uint64)
        _check(self.lib.kc_server_read_distinct(self._h, int(session), int(first), int(n),
                                                out.ctypes.data), "kc_server_read_distinct")
        return out[:int(n)]

    def read_words(self, session: int, n_words: int):
        import numpy as np
        out = np.zeros(int(n_words), dtype=np.uint64)
        _check(self.lib.kc_server_read_words(self._h, int(session), out.ctypes.data),
               "kc_server_read_words")
        return out

    def stats(self) -> dict:
        st = kc_server_stats()
        _check(self.lib.kc_server_stats_get(self._h, ctypes.byref(st)), "kc_server_stats_get")
        return {f: getattr(st, f) for f, _ in kc_server_stats._fields_}

    def now(self) -> float:
        return float(self.lib.kc_server_now(self._h))
