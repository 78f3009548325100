"""KmerCo CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes + numpy) to the plain single-threaded C oracle in
``kmerco_oracle.c``.  Only the tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library never imports, links or calls it.

Parity status of each function (how it is pinned, see ``tests/test_oracle_*``):
  mm3_32      library: scikit-learn's MurmurHash3_x86_32
  revcomp     paper's worked example (Sec. 2.2) + brute-force involution
  encode      definition on hand-checked strings
  dims        all nine countBF sizes printed in the paper (Fig. 4 data,
              supplement size table)
  eta         supplement counter-length table
  insert      paper's window count (Sec. 1.1); counters == min(max, bincount)
              of the occurrences' slots (numpy); distinct == first occurrence
              per slot (numpy.unique) for k_h = 1; exact brute-force counts and
              first-seen order when the filter has no collisions; strand
              symmetry; incremental == concatenated
  query       exact counts when collision-free; >= exact count always
  classify    partition of the distinct list; one-sided error vs exact counts
  *_wide      K = 33..64 (128-bit keys): the same pins with brute force on
              Python strings and scikit-learn's MurmurHash3 of the 16-byte key
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmerco_oracle.c")
_LIB = os.path.join(_HERE, "libkmerco_oracle.so")

OK, EINVAL, ERANGE = 0, -1, -3


class Layout(ctypes.Structure):
    _fields_ = [("X", ctypes.c_uint64), ("Y", ctypes.c_uint64),
                ("alpha", ctypes.c_uint32), ("k_h", ctypes.c_uint32)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lp = ctypes.POINTER(Layout)
        L.kco_mm3_32.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32]
        L.kco_mm3_32.restype = ctypes.c_uint32
        L.kco_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.kco_hash.restype = ctypes.c_uint64
        L.kco_revcomp.argtypes = [u8p, ctypes.c_uint64, u8p]
        L.kco_revcomp.restype = None
        L.kco_encode.argtypes = [u8p, ctypes.c_uint32, u64p]
        L.kco_encode.restype = ctypes.c_int
        L.kco_eta.argtypes = [ctypes.c_uint32]
        L.kco_eta.restype = ctypes.c_uint32
        L.kco_slot.argtypes = [lp, ctypes.c_uint64, u64p, u32p]
        L.kco_slot.restype = None
        L.kco_query.argtypes = [lp, u64p, ctypes.c_uint64]
        L.kco_query.restype = ctypes.c_uint64
        L.kco_canonical.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.kco_canonical.restype = ctypes.c_uint64
        L.kco_insert.argtypes = [lp, u64p, u8p, u64p, ctypes.c_uint64, ctypes.c_uint32,
                                 u64p, ctypes.c_uint64, u64p, u64p]
        L.kco_insert.restype = ctypes.c_int
        L.kco_classify.argtypes = [lp, u64p, u64p, ctypes.c_uint64, ctypes.c_uint64,
                                   u64p, u64p, u64p, u64p]
        L.kco_classify.restype = ctypes.c_int
        L.kco_query_many.argtypes = [lp, u64p, u64p, ctypes.c_uint64, u64p]
        L.kco_query_many.restype = ctypes.c_int
        L.kco_occurrences.argtypes = [lp, u8p, u64p, ctypes.c_uint64, ctypes.c_uint32,
                                      u64p, u64p, ctypes.c_uint64, u64p]
        L.kco_occurrences.restype = ctypes.c_int
        L.kco_hash_wide.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.kco_hash_wide.restype = ctypes.c_uint64
        L.kco_query_wide.argtypes = [lp, u64p, ctypes.c_uint64, ctypes.c_uint64]
        L.kco_query_wide.restype = ctypes.c_uint64
        L.kco_insert_wide.argtypes = L.kco_insert.argtypes
        L.kco_insert_wide.restype = ctypes.c_int
        L.kco_classify_wide.argtypes = L.kco_classify.argtypes
        L.kco_classify_wide.restype = ctypes.c_int
        L.kco_occurrences_wide.argtypes = L.kco_occurrences.argtypes
        L.kco_occurrences_wide.restype = ctypes.c_int
        L.kco_dims.argtypes = [ctypes.c_double, ctypes.c_double, u64p, u64p]
        L.kco_dims.restype = ctypes.c_int
        L.kco_is_prime.argtypes = [ctypes.c_uint64]
        L.kco_is_prime.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, _p(a, ctypes.c_uint8)


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, _p(a, ctypes.c_uint64)


# ---------------------------------------------------------------------------
# scalar helpers
# ---------------------------------------------------------------------------

def mm3_32(data: bytes, seed: int) -> int:
    buf = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)  # never empty
    return int(lib().kco_mm3_32(_p(buf, ctypes.c_uint8), len(data), seed))


def hash_a(key: int, a: int, k: int = 32) -> int:
    """H_a of a 2-bit key; keys of k > 32 bases (reading R15) as 16 bytes."""
    if k > 32:
        return int(lib().kco_hash_wide(key & ((1 << 64) - 1), key >> 64, a))
    return int(lib().kco_hash(key, a))


def pairs_to_ints(a) -> list:
    """(n, 2) uint64 (low, high) key pairs -> Python ints."""
    a = np.asarray(a, dtype=np.uint64).reshape(-1, 2)
    return [int(lo) | (int(hi) << 64) for lo, hi in a]


def revcomp(s: bytes) -> bytes:
    src = np.frombuffer(bytes(s) + b"\0", dtype=np.uint8)
    out = np.zeros(len(s) + 1, dtype=np.uint8)
    lib().kco_revcomp(_p(src, ctypes.c_uint8), len(s), _p(out, ctypes.c_uint8))
    return out[:len(s)].tobytes()


def encode(s: bytes):
    """2-bit key of s (first base most significant), or None if invalid."""
    src = np.frombuffer(bytes(s) + b"\0", dtype=np.uint8)
    v = ctypes.c_uint64(0)
    rc = lib().kco_encode(_p(src, ctypes.c_uint8), len(s), ctypes.byref(v))
    return None if rc != 0 else int(v.value)


def canonical(fwd: int, rc: int) -> int:
    return int(lib().kco_canonical(fwd, rc))


def eta(alpha: int) -> int:
    return int(lib().kco_eta(alpha))


def is_prime(n: int) -> bool:
    return bool(lib().kco_is_prime(n))


def dims(n_items: float, fpp: float = 0.001):
    X = ctypes.c_uint64(0)
    Y = ctypes.c_uint64(0)
    rc = lib().kco_dims(float(n_items), float(fpp), ctypes.byref(X), ctypes.byref(Y))
    if rc != OK:
        raise ValueError(f"kco_dims failed ({rc})")
    return int(X.value), int(Y.value)


def slot(X: int, Y: int, alpha: int, h: int):
    L = Layout(X, Y, alpha, 1)
    w = ctypes.c_uint64(0)
    l = ctypes.c_uint32(0)
    lib().kco_slot(ctypes.byref(L), h, ctypes.byref(w), ctypes.byref(l))
    return int(w.value), int(l.value)


# ---------------------------------------------------------------------------
# the countBF
# ---------------------------------------------------------------------------

class CountBF:
    """A countBF held in host memory and driven by the oracle."""

    def __init__(self, X: int, Y: int, alpha: int = 8, k_h: int = 1):
        self.layout = Layout(X, Y, alpha, k_h)
        self.words = np.zeros(X * Y, dtype=np.uint64)
        self.k = None

    @property
    def eta(self):
        return eta(self.layout.alpha)

    def insert(self, reads, offsets, k: int):
        """Algorithm 1 over one read batch; returns (distinct keys, n_windows).
        Keys of k > 32 bases come as an (n, 2) array of (low, high) words."""
        reads, rp = _u8(reads)
        offsets, op = _u64(offsets)
        n_reads = len(offsets) - 1
        cap = max(1, int(offsets[-1]) if n_reads > 0 else 1)
        w = 2 if k > 32 else 1
        out = np.zeros(cap * w, dtype=np.uint64)
        nd = ctypes.c_uint64(0)
        nw = ctypes.c_uint64(0)
        fn = lib().kco_insert_wide if k > 32 else lib().kco_insert
        rc = fn(ctypes.byref(self.layout), _p(self.words, ctypes.c_uint64), rp, op,
                n_reads, k, _p(out, ctypes.c_uint64), cap, ctypes.byref(nd), ctypes.byref(nw))
        if rc != OK:
            raise ValueError(f"kco_insert failed ({rc})")
        self.k = k
        d = out[:nd.value * w].copy()
        return (d.reshape(-1, 2) if w == 2 else d), int(nw.value)

    def query(self, keys):
        if np.ndim(keys) == 2:  # (low, high) pairs of k > 32 keys
            L = lib()
            w = _p(self.words, ctypes.c_uint64)
            return np.array([L.kco_query_wide(ctypes.byref(self.layout), w, int(lo), int(hi))
                             for lo, hi in np.asarray(keys, dtype=np.uint64)], dtype=np.uint64)
        keys, kp = _u64(keys)
        out = np.zeros(max(1, len(keys)), dtype=np.uint64)
        rc = lib().kco_query_many(ctypes.byref(self.layout), _p(self.words, ctypes.c_uint64),
                                  kp, len(keys), _p(out, ctypes.c_uint64))
        if rc != OK:
            raise ValueError(f"kco_query_many failed ({rc})")
        return out[:len(keys)]

    def classify(self, distinct, tau: int):
        """Algorithm 2; (n, 2) key pairs (k > 32) give (n, 2) outputs."""
        wide = np.ndim(distinct) == 2
        distinct, dp = _u64(distinct)
        w = 2 if wide else 1
        n = distinct.size // w
        trust = np.zeros(max(1, n) * w, dtype=np.uint64)
        err = np.zeros(max(1, n) * w, dtype=np.uint64)
        nt = ctypes.c_uint64(0)
        ne = ctypes.c_uint64(0)
        fn = lib().kco_classify_wide if wide else lib().kco_classify
        rc = fn(ctypes.byref(self.layout), _p(self.words, ctypes.c_uint64), dp, n, tau,
                _p(trust, ctypes.c_uint64), ctypes.byref(nt), _p(err, ctypes.c_uint64),
                ctypes.byref(ne))
        if rc != OK:
            raise ValueError(f"kco_classify failed ({rc})")
        t, e = trust[:nt.value * w].copy(), err[:ne.value * w].copy()
        return (t.reshape(-1, 2), e.reshape(-1, 2)) if wide else (t, e)

    def counters(self):
        """Unpacked counters, shape (X*Y, eta), counter l of word w at [w, l]."""
        a = self.layout.alpha
        e = self.eta
        mask = np.uint64((1 << a) - 1) if a < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        cols = [(self.words >> np.uint64(a * l)) & mask for l in range(e)]
        return np.stack(cols, axis=1)


def occurrences(reads, offsets, k: int, X: int, Y: int, alpha: int = 8, k_h: int = 1):
    """Canonical k-mer and slot ids (word*eta + l, one per hash function) of
    every valid window, in Algorithm 1's order."""
    reads, rp = _u8(reads)
    offsets, op = _u64(offsets)
    n_reads = len(offsets) - 1
    cap = max(1, int(offsets[-1]))
    kmers = np.zeros(cap, dtype=np.uint64)
    slots = np.zeros(cap * k_h, dtype=np.uint64)
    n = ctypes.c_uint64(0)
    L = Layout(X, Y, alpha, k_h)
    if k > 32:
        kmers = np.zeros(cap * 2, dtype=np.uint64)
    fn = lib().kco_occurrences_wide if k > 32 else lib().kco_occurrences
    rc = fn(ctypes.byref(L), rp, op, n_reads, k, _p(kmers, ctypes.c_uint64),
            _p(slots, ctypes.c_uint64), cap, ctypes.byref(n))
    if rc != OK:
        raise ValueError(f"kco_occurrences failed ({rc})")
    m = int(n.value)
    km = kmers[:m * 2].reshape(m, 2).copy() if k > 32 else kmers[:m].copy()
    return km, slots[:m * k_h].reshape(m, k_h).copy()


def run_kmerco(reads, offsets, k: int, tau: int, X: int, Y: int, alpha: int = 8, k_h: int = 1):
    """Both phases on a fresh countBF: (words, distinct, trustworthy, erroneous, n_windows)."""
    bf = CountBF(X, Y, alpha, k_h)
    distinct, nw = bf.insert(reads, offsets, k)
    trust, err = bf.classify(distinct, tau)
    return bf.words, distinct, trust, err, nw
