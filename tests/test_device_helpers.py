"""CPU checks of the GPU path's arithmetic (compiled for the host from the
same header the kernels use): exact Barrett reduction, the packed window
layout, 2-bit reverse complement, MurmurHash3 and the canonical choice."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
from sklearn.utils import murmurhash3_32

from tests import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_07545_amd", "csrc")


@pytest.fixture(scope="module")
def H(tmp_path_factory):
    out = tmp_path_factory.mktemp("kch") / "libkch.so"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-fPIC", "-shared", "-I", CSRC,
                           os.path.join(ROOT, "tests", "device_helpers_host.hip"), "-o", str(out)],
                          stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(str(out))
    u64, u32 = ctypes.c_uint64, ctypes.c_uint32
    p32 = ctypes.POINTER(ctypes.c_uint32)
    L.kch_mod_by.argtypes = [u64, u64]; L.kch_mod_by.restype = u64
    L.kch_mod_small.argtypes = [u64, u32]; L.kch_mod_small.restype = u64
    L.kch_mod_small_mismatches.argtypes = [u32, u64, u64]
    L.kch_mod_small_mismatches.restype = u64
    L.kch_codes4.argtypes = [u32, ctypes.POINTER(u32)]; L.kch_codes4.restype = u32
    L.kch_revcomp.argtypes = [u64, u32]; L.kch_revcomp.restype = u64
    L.kch_window_key.argtypes = [p32, u64, u32]; L.kch_window_key.restype = u64
    L.kch_window_valid.argtypes = [p32, p32, p32, u64, u32, u64]; L.kch_window_valid.restype = ctypes.c_int
    L.kch_hash.argtypes = [u64, u32]; L.kch_hash.restype = u64
    L.kch_valid_word.argtypes = [p32, p32, u64, u64, u32, u64]; L.kch_valid_word.restype = u32
    L.kch_wave_valid.argtypes = [p32, u64]; L.kch_wave_valid.restype = u64
    L.kch_canonical.argtypes = [u64, u32, ctypes.POINTER(u64)]; L.kch_canonical.restype = u64
    L.kch_slot.argtypes = [u64, u64, u32, u64, ctypes.POINTER(u64), ctypes.POINTER(u32)]
    L.kch_slot.restype = None
    L.kch_base.argtypes = [u32, ctypes.POINTER(u32)]; L.kch_base.restype = ctypes.c_int
    L.kch_wave_window.argtypes = [p32, p32, p32, u64, u32, u64, ctypes.POINTER(u64)]
    L.kch_wave_window.restype = ctypes.c_int
    pu64 = ctypes.POINTER(u64)
    L.kch_window_key_wide.argtypes = [p32, u64, u32, pu64, pu64]
    L.kch_window_key_wide.restype = None
    L.kch_revcomp_wide.argtypes = [u64, u64, u32, pu64, pu64]
    L.kch_revcomp_wide.restype = None
    L.kch_hash_wide.argtypes = [u64, u64, u32]
    L.kch_hash_wide.restype = u64
    L.kch_canonical_wide.argtypes = [u64, u64, u32, pu64, pu64, pu64]
    L.kch_canonical_wide.restype = None
    L.kch_canonical_fast.argtypes = [u64, u32, ctypes.POINTER(u64)]
    L.kch_canonical_fast.restype = u64
    return L


def test_mod_by_exact(H):
    rng = np.random.default_rng(1)
    ds = [1, 2, 3, 7, 8, 12, 13, 239, 257, 2621, 2657, 31627, 31657, 2**31 - 1, 2**32 + 15,
          2**40 + 7, 2**63 + 25, 2**64 - 1]
    hs = [0, 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1, 2**64 - 2]
    hs += [int(x) for x in rng.integers(0, 2**63, 300, dtype=np.int64)]
    hs += [int(x) * 2 + 1 for x in rng.integers(0, 2**63, 300, dtype=np.int64)]
    for d in ds:
        for h in hs + [d * 5, d * 5 - 1, (2**64 - 1) // d * d, (2**64 - 1) // d * d - 1]:
            h %= 2**64
            assert H.kch_mod_by(h, d) == h % d, (h, d)


SMALL_MAX = (2**32 - 1) // 3


def test_mod_small_exact(H):
    """The 32-bit reduction for divisors up to (2^32-1)/3: exact remainders on
    edge values, near multiples of d and a million pseudo-random values per
    divisor."""
    rng = np.random.default_rng(4)
    ds = [1, 2, 3, 5, 8, 239, 2621, 2657, 31627, 65536, 2**20 + 7, 2**30, 2**30 + 3,
          SMALL_MAX - 1, SMALL_MAX] + [int(x) for x in rng.integers(1, SMALL_MAX, 12)]
    for d in ds:
        edge = [0, 1, d - 1, d, d + 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1, 2**64 - 2,
                (2**64 - 1) // d * d, (2**64 - 1) // d * d - 1]
        for h in edge:
            h %= 2**64
            assert H.kch_mod_small(h, d) == h % d, (h, d)
        assert H.kch_mod_small_mismatches(d, 1 << 20, 17 + d) == 0, d


def test_slot_map(H):
    rng = np.random.default_rng(2)
    for X, Y, alpha in [(239, 257, 8), (3, 5, 5), (2621, 2657, 7), (31627, 31657, 12),
                        (1, 1, 32), (13, 17, 3), (SMALL_MAX, SMALL_MAX - 2, 8),
                        (SMALL_MAX + 1, 7, 8), (5, 2**33 + 1, 16)]:
        eta = 64 // alpha
        for h in [0, 2**64 - 1] + [int(x) * 3 for x in rng.integers(0, 2**62, 200, dtype=np.int64)]:
            w = ctypes.c_uint64()
            l = ctypes.c_uint32()
            H.kch_slot(X, Y, alpha, h, ctypes.byref(w), ctypes.byref(l))
            assert (w.value, l.value) == ((h % X) * Y + (h % Y), h % eta)


def test_codes4_every_byte_in_every_lane(H):
    """The 4-bases-at-a-time conversion: every byte value in each of the 4
    lanes, beside random neighbours, against the one-base definition."""
    rng = np.random.default_rng(6)
    v = ctypes.c_uint32()
    c = ctypes.c_uint32()
    for lane in range(4):
        for b in range(256):
            others = [int(x) for x in rng.integers(0, 256, 3)]
            others.insert(lane, b)
            x = sum(o << (8 * i) for i, o in enumerate(others))
            got = H.kch_codes4(x, ctypes.byref(v))
            want_c, want_v = 0, 0
            for i, o in enumerate(others):
                ok = H.kch_base(o, ctypes.byref(c))
                want_v |= ok << i
                want_c |= (c.value if ok else 0) << (6 - 2 * i)
            assert (got, v.value) == (want_c, want_v), (hex(x), lane, b)
    for x in [0, 0xFFFFFFFF, 0x54474341, 0x41414141, 0x54545454, 0x4E4E4E4E, 0x80C1C3C7]:
        got = H.kch_codes4(x, ctypes.byref(v))
        want_c, want_v = 0, 0
        for i in range(4):
            o = (x >> (8 * i)) & 0xFF
            ok = H.kch_base(o, ctypes.byref(c))
            want_v |= ok << i
            want_c |= (c.value if ok else 0) << (6 - 2 * i)
        assert (got, v.value) == (want_c, want_v), hex(x)


def test_base_codes(H):
    c = ctypes.c_uint32()
    for b in range(256):
        ok = H.kch_base(b, ctypes.byref(c))
        if chr(b) in "ACGT":
            assert ok == 1 and c.value == "ACGT".index(chr(b))
        else:
            assert ok == 0, chr(b)


def test_hash_matches_library(H):
    rng = np.random.default_rng(3)
    for key in [0, 1, 2**64 - 1] + [int(x) for x in rng.integers(0, 2**63, 200, dtype=np.int64)]:
        for a in (1, 2, 5, 8):
            assert H.kch_hash(key, a) == brute.h64(key, a)


def test_revcomp_and_canonical(H):
    rng = np.random.default_rng(4)
    for K in (1, 2, 3, 15, 16, 21, 31, 32):
        for _ in range(60):
            s = "".join(rng.choice(list("ACGT"), size=K))
            f = brute.key_of(s)
            r = brute.key_of(brute.revcomp_str(s))
            assert H.kch_revcomp(f, K) == r
            h1 = ctypes.c_uint64()
            assert H.kch_canonical(f, K, ctypes.byref(h1)) == brute.canonical_str(s)
            assert h1.value == min(brute.h64(f), brute.h64(r)) or f == r
            h1f = ctypes.c_uint64()
            assert H.kch_canonical_fast(f, K, ctypes.byref(h1f)) == brute.canonical_str(s)
            assert h1f.value == h1.value


def _pack(seq: bytes, starts):
    """The packed layout written by the ingest kernel, built here from its
    documented definition: 16 bases per code word (first base in bits
    31..30), 32 bases per mask word (bit q%32), padding invalid."""
    n = len(seq)
    tiles = (n + 1023) // 1024
    codes = np.zeros(tiles * 64 + 4, dtype=np.uint32)
    inv = np.zeros(tiles * 32 + 2, dtype=np.uint32)
    rs = np.zeros(tiles * 32 + 2, dtype=np.uint32)
    for q in range(len(inv) * 32):
        ch = chr(seq[q]) if q < n else "?"
        if ch in "ACGT":
            codes[q // 16] |= np.uint32("ACGT".index(ch) << (30 - 2 * (q % 16)))
        else:
            inv[q // 32] |= np.uint32(1 << (q % 32))
    for o in starts:
        if o < n:
            rs[o // 32] |= np.uint32(1 << (o % 32))
    return codes, inv, rs


def test_window_extraction_matches_brute_force(H):
    rng = np.random.default_rng(5)
    reads = []
    for _ in range(40):
        ln = int(rng.integers(0, 90))
        reads.append("".join(rng.choice(list("ACGTNa"), p=[.24, .24, .24, .24, .02, .02], size=ln)))
    buf = "".join(reads).encode()
    starts = np.cumsum([0] + [len(r) for r in reads])[:-1]
    codes, inv, rs = _pack(buf, starts)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))  # noqa: E731
    for K in (1, 5, 16, 21, 31, 32):
        valid = set()
        for r, o in zip(reads, starts):
            for p in range(len(r) - K + 1):
                if all(c in "ACGT" for c in r[p:p + K]):
                    valid.add(int(o) + p)
        for p in range(len(buf)):
            v = H.kch_window_valid(P(codes), P(inv), P(rs), len(buf), K, p)
            assert v == (p in valid), (K, p)
            if v:
                assert H.kch_window_key(P(codes), p, K) == brute.key_of(buf[p:p + K].decode())
            fw = ctypes.c_uint64()
            wv = H.kch_wave_window(P(codes), P(inv), P(rs), len(buf), K, p, ctypes.byref(fw))
            assert wv == v, (K, p)
            if v:
                assert fw.value == brute.key_of(buf[p:p + K].decode())


def test_valid_window_bitmap_matches_brute_force(H):
    """The valid-window bitmap the binned paths read (bit p: the K-base
    window at p is inside one read and holds only A, C, G, T), for short and
    long K, against Python strings; and the 64-bit word a wavefront takes."""
    rng = np.random.default_rng(25)
    reads = []
    for _ in range(60):
        ln = int(rng.integers(0, 160))
        reads.append("".join(rng.choice(list("ACGTNa"), p=[.2425, .2425, .2425, .2425, .02, .01],
                                        size=ln)))
    buf = "".join(reads).encode()
    starts = np.cumsum([0] + [len(r) for r in reads])[:-1]
    _, inv, rs = _pack(buf, starts)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))  # noqa: E731
    n_words = len(inv)
    for K in (1, 2, 5, 16, 21, 31, 32, 33, 40, 55, 63, 64):
        valid = set()
        for r, o in zip(reads, starts):
            for p in range(len(r) - K + 1):
                if all(c in "ACGT" for c in r[p:p + K]):
                    valid.add(int(o) + p)
        bits = np.array([H.kch_valid_word(P(inv), P(rs), n_words, i, K, len(buf))
                         for i in range(n_words)], dtype=np.uint32)
        got = {32 * i + j for i in range(n_words) for j in range(32) if (int(bits[i]) >> j) & 1}
        assert got == valid, (K, sorted(got ^ valid)[:10])
        for pb in range(0, 32 * (n_words - 1), 64):
            want = sum(1 << (p - pb) for p in valid if pb <= p < pb + 64)
            assert H.kch_wave_valid(P(bits), pb) == want, (K, pb)


def _wide(lo, hi):
    return int(lo) | (int(hi) << 64)


def test_wide_window_extraction_matches_brute_force(H):
    """Keys of 33..64 bases from the packed layout: the 128-bit key of every
    valid window, against Python strings (validity: the bitmap test)."""
    rng = np.random.default_rng(15)
    reads = []
    for _ in range(25):
        ln = int(rng.integers(0, 200))
        reads.append("".join(rng.choice(list("ACGTN"), p=[.245, .245, .245, .245, .02], size=ln)))
    buf = "".join(reads).encode()
    starts = np.cumsum([0] + [len(r) for r in reads])[:-1]
    codes, inv, rs = _pack(buf, starts)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))  # noqa: E731
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    for K in (33, 40, 55, 63, 64):
        valid = set()
        for r, o in zip(reads, starts):
            for p in range(len(r) - K + 1):
                if all(c in "ACGT" for c in r[p:p + K]):
                    valid.add(int(o) + p)
        for p in sorted(valid):
            H.kch_window_key_wide(P(codes), p, K, ctypes.byref(lo), ctypes.byref(hi))
            assert _wide(lo.value, hi.value) == brute.key_of(buf[p:p + K].decode()), (K, p)


def test_wide_revcomp_hash_canonical(H):
    rng = np.random.default_rng(16)
    lo, hi, h1 = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    for K in (33, 47, 55, 64):
        for _ in range(60):
            s = "".join(rng.choice(list("ACGT"), size=K))
            key = brute.key_of(s)
            k_lo, k_hi = key & ((1 << 64) - 1), key >> 64
            H.kch_revcomp_wide(k_lo, k_hi, K, ctypes.byref(lo), ctypes.byref(hi))
            assert _wide(lo.value, hi.value) == brute.key_of(brute.revcomp_str(s))
            for a in (1, 2, 8):
                assert H.kch_hash_wide(k_lo, k_hi, a) == brute.h64(key, a, 16)
            H.kch_canonical_wide(k_lo, k_hi, K, ctypes.byref(lo), ctypes.byref(hi),
                                 ctypes.byref(h1))
            c = brute.canonical_str(s)
            assert _wide(lo.value, hi.value) == c
            assert h1.value == brute.h64(c, 1, 16)

