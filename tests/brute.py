"""Brute-force k-mer facts for tiny inputs, computed directly from the paper's
definitions with Python strings and scikit-learn's MurmurHash3 (a library
routine independent of the C oracle).  Used only to pin the oracle."""
from __future__ import annotations

from collections import OrderedDict

from sklearn.utils import murmurhash3_32

_COMP = str.maketrans("ACGTN", "TGCAN")
_DIGIT = str.maketrans("ACGT", "0123")


def revcomp_str(s: str) -> str:
    """Sec. 2.2: complement each base, then reverse."""
    return s.translate(_COMP)[::-1]


def key_of(s: str) -> int:
    """2-bit key, first base most significant."""
    return int(s.translate(_DIGIT), 4)


def h64(key: int, a: int = 1, nbytes: int = 8) -> int:
    """H_a: two 32-bit MurmurHash3_x86_32 values of the little-endian key
    (8 bytes for K <= 32; 16 bytes for K = 33..64)."""
    b = key.to_bytes(nbytes, "little")
    hi = murmurhash3_32(b, seed=2 * a - 2, positive=True)
    lo = murmurhash3_32(b, seed=2 * a - 1, positive=True)
    return (hi << 32) | lo


def canonical_str(window: str) -> int:
    """Sec. 2.3: the strand whose hash is smaller (ties: reverse complement)."""
    f = key_of(window)
    r = key_of(revcomp_str(window))
    nb = 16 if len(window) > 32 else 8
    return f if h64(f, 1, nb) < h64(r, 1, nb) else r


def windows(reads: list[str], k: int):
    """Every valid window (only A/C/G/T, inside one read), in read order and
    increasing start position."""
    for s in reads:
        for p in range(len(s) - k + 1):
            w = s[p:p + k]
            if all(c in "ACGT" for c in w):
                yield w


def exact_counts(reads: list[str], k: int) -> "OrderedDict[int, int]":
    """Exact canonical k-mer counts, keys in first-occurrence order."""
    counts: OrderedDict[int, int] = OrderedDict()
    for w in windows(reads, k):
        c = canonical_str(w)
        counts[c] = counts.get(c, 0) + 1
    return counts


def split_reads(rs) -> list[str]:
    """A synth.ReadSet as a list of Python strings."""
    buf = rs.reads.tobytes()
    o = [int(x) for x in rs.offsets]
    return [buf[o[i]:o[i + 1]].decode("latin-1") for i in range(len(o) - 1)]
