"""Pins of the CPU oracle against things other than itself: values printed in
the paper, a library MurmurHash3, closed forms, invariants and brute force.

Each test names the paper passage it checks."""
import json
import os

import numpy as np
import pytest
import sympy
from sklearn.utils import murmurhash3_32

import synth
from tests import brute

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# --------------------------------------------------------------------------
# hash (reading: MurmurHash3_x86_32, the murmur hash named in Sec. 3)
# --------------------------------------------------------------------------

def test_mm3_matches_library(oracle_lib):
    rng = np.random.default_rng(7)
    for ln in list(range(0, 20)) + [31, 32, 33, 64]:
        for seed in (0, 1, 2, 3, 15, 0x9747B28C, 0xFFFFFFFF):
            b = rng.integers(0, 256, ln, dtype=np.uint8).tobytes()
            assert oracle_lib.mm3_32(b, seed) == murmurhash3_32(b, seed=seed, positive=True)


def test_hash_a_is_two_mm3_words(oracle_lib):
    rng = np.random.default_rng(8)
    keys = [0, 1, 2**62 - 1, 2**64 - 1] + [int(x) for x in rng.integers(0, 2**63, 50, dtype=np.int64)]
    for key in keys:
        for a in (1, 2, 3, 8):
            assert oracle_lib.hash_a(key, a) == brute.h64(key, a)


# --------------------------------------------------------------------------
# sequences (Sec. 1.1 k-mers, Sec. 2.2 reverse complement)
# --------------------------------------------------------------------------

def test_revcomp_paper_example(oracle_lib):
    ex = GOLDEN["revcomp_example"]
    assert oracle_lib.revcomp(ex["sequence"].encode()) == ex["reverse_complement"].encode()
    # complement alone = reverse of the reverse complement
    assert oracle_lib.revcomp(ex["sequence"].encode())[::-1] == ex["complement"].encode()
    # N stays N (Sec. 2.2)
    assert oracle_lib.revcomp(b"ANGT") == b"ACNT"


def test_revcomp_involution_brute(oracle_lib):
    rng = np.random.default_rng(9)
    for _ in range(200):
        s = bytes(rng.choice(list(b"ACGTN"), size=int(rng.integers(1, 40))))
        r = oracle_lib.revcomp(s)
        assert r == brute.revcomp_str(s.decode()).encode()
        assert oracle_lib.revcomp(r) == s


def test_encode_definition(oracle_lib):
    assert oracle_lib.encode(b"A" * 21) == 0
    assert oracle_lib.encode(b"T" * 32) == 2**64 - 1
    assert oracle_lib.encode(b"ACGT") == 0b00011011
    assert oracle_lib.encode(b"CA") == 4
    assert oracle_lib.encode(b"ACNT") is None
    assert oracle_lib.encode(b"acgt") is None


def test_window_count_paper_example(oracle_lib):
    ex = GOLDEN["kmer_example"]
    seq, K = ex["sequence"], ex["K"]
    rs = synth.reads_from_strings([seq], k=K)
    kmers, slots = oracle_lib.occurrences(rs.reads, rs.offsets, K, 101, 107)
    assert len(kmers) == len(seq) - K + 1 == len(ex["kmers"])
    for got, w in zip(kmers, ex["kmers"]):
        assert int(got) in (brute.key_of(w), brute.key_of(brute.revcomp_str(w)))
    bf = oracle_lib.CountBF(101, 107)
    _, nw = bf.insert(rs.reads, rs.offsets, K)
    assert nw == 6
    assert int(bf.counters().sum()) == 6


# --------------------------------------------------------------------------
# countBF layout (Sec. 2.1) and sizing (Eq. 1)
# --------------------------------------------------------------------------

def test_counter_table(oracle_lib):
    for alpha, eta, wasted in GOLDEN["counter_table"]["rows"]:
        assert oracle_lib.eta(alpha) == eta
        assert 64 - alpha * oracle_lib.eta(alpha) == wasted


def _mib(X, Y):
    return X * Y * 8 / 2**20


def _matches_printed(value, printed: str):
    decimals = len(printed.split(".")[1]) if "." in printed else 0
    return abs(value - float(printed)) < 10.0 ** (-decimals)


def test_dims_reproduce_printed_sizes(oracle_lib):
    """All nine printed countBF sizes come out of Eq. (1) evaluated at n/2
    (the reading recorded for the sizing formula)."""
    for row in GOLDEN["countbf_sizes"]["rows"]:
        X, Y = oracle_lib.dims(row["n"] / 2, 0.001)
        assert sympy.isprime(X) and sympy.isprime(Y)
        assert Y == sympy.nextprime(sympy.nextprime(sympy.nextprime(X)))
        assert X == sympy.nextprime(int(np.floor(np.sqrt(-row["n"] / 2 * np.log(0.001)
                                                         / np.log(2) ** 2 / 128))))
        assert _matches_printed(_mib(X, Y), row["size"]), (row, X, Y, _mib(X, Y))


def test_dims_pin_discriminates(oracle_lib):
    """Taking the 2nd prime after X, or n instead of n/2, misses printed sizes."""
    misses_second = 0
    misses_full = 0
    for row in GOLDEN["countbf_sizes"]["rows"]:
        X, _ = oracle_lib.dims(row["n"] / 2, 0.001)
        Y2 = sympy.nextprime(sympy.nextprime(X))
        misses_second += not _matches_printed(_mib(X, Y2), row["size"])
        Xf, Yf = oracle_lib.dims(row["n"], 0.001)
        misses_full += not _matches_printed(_mib(Xf, Yf), row["size"])
    assert misses_second >= 4
    assert misses_full == len(GOLDEN["countbf_sizes"]["rows"])


def test_dims_errors(oracle_lib):
    for bad in [(0, 0.001), (10, 0.0), (10, 1.0), (-5, 0.01)]:
        with pytest.raises(ValueError):
            oracle_lib.dims(*bad)


def test_ins_per_second_definition():
    ex = GOLDEN["insertions_per_second"]
    assert abs(ex["insertions"] / ex["seconds"] - ex["per_second"]) < 1e-3


# --------------------------------------------------------------------------
# countBF insert / query (Algorithms 3, 4, 5)
# --------------------------------------------------------------------------

def test_single_kmer_placement(oracle_lib):
    """One window sets exactly counter l of word i*Y + j to 1, with i, j, l
    taken from H_1 of the canonical strand (Algorithm 3), and counter 0 sits
    at the low byte (the first extract mask of Sec. 2.1)."""
    rng = np.random.default_rng(10)
    X, Y = 251, 263
    for _ in range(40):
        s = "".join(rng.choice(list("ACGT"), size=25))
        rs = synth.reads_from_strings([s], k=25)
        bf = oracle_lib.CountBF(X, Y, 8, 1)
        d, nw = bf.insert(rs.reads, rs.offsets, 25)
        c = brute.canonical_str(s)
        h = brute.h64(c, 1)
        i, j, l = h % X, h % Y, h % 8
        expect = np.zeros(X * Y, dtype=np.uint64)
        expect[i * Y + j] = np.uint64(1) << np.uint64(8 * l)
        assert np.array_equal(bf.words, expect)
        assert list(d) == [c] and nw == 1
    ext = int(GOLDEN["masks_alpha8"]["extract_first"], 16)
    assert (1 << 8) - 1 == ext


@pytest.mark.parametrize("alpha,k_h", [(8, 1), (8, 2), (8, 3), (4, 1), (5, 2), (16, 1), (12, 3)])
def test_counters_are_saturated_slot_counts(oracle_lib, alpha, k_h):
    """Closed form: every counter equals min(2^alpha - 1, number of
    (occurrence, hash function) pairs that map to it) -- numpy.bincount."""
    rs = synth.random_reads(11 + alpha + k_h, 60, 20, 90, k=9, alphabet=b"ACGT", p_n=0.02)
    X, Y = 13, 17  # tiny filter: many collisions
    bf = oracle_lib.CountBF(X, Y, alpha, k_h)
    _, nw = bf.insert(rs.reads, rs.offsets, 9)
    kmers, slots = oracle_lib.occurrences(rs.reads, rs.offsets, 9, X, Y, alpha, k_h)
    assert len(kmers) == nw
    eta = oracle_lib.eta(alpha)
    hits = np.bincount(slots.ravel().astype(np.int64), minlength=X * Y * eta)
    expect = np.minimum(hits, (1 << alpha) - 1).reshape(X * Y, eta)
    assert np.array_equal(bf.counters().astype(np.int64), expect)
    # Query-II (Algorithm 5) = the minimum of the k_h counters of the k-mer
    q = bf.query(kmers).astype(np.int64)
    assert np.array_equal(q, expect.ravel()[slots.astype(np.int64)].min(axis=1))
    # bits above eta*alpha stay zero
    used = alpha * eta
    if used < 64:
        assert not np.any(bf.words >> np.uint64(used))


@pytest.mark.parametrize("k_h", [1, 2, 3])
def test_distinct_is_first_occurrence_per_slot(oracle_lib, k_h):
    """Algorithm 1 with Query-I: an occurrence is distinct iff, for some hash
    function, it is the first occurrence to touch that slot -- numpy.unique's
    first indices on the flattened (occurrence, hash fn) slot list."""
    rs = synth.random_reads(21 + k_h, 80, 15, 60, k=7, alphabet=b"ACGT")
    X, Y = 11, 19
    bf = oracle_lib.CountBF(X, Y, 8, k_h)
    distinct, _ = bf.insert(rs.reads, rs.offsets, 7)
    kmers, slots = oracle_lib.occurrences(rs.reads, rs.offsets, 7, X, Y, 8, k_h)
    _, first = np.unique(slots.ravel(), return_index=True)
    occ = np.unique(first // k_h)
    assert np.array_equal(distinct, kmers[occ])
    if k_h == 1:
        assert len(distinct) == int(np.count_nonzero(bf.counters()))


def test_collision_free_exact(oracle_lib):
    """With a filter far larger than the k-mer set (and no slot shared between
    distinct k-mers), KmerCo is exact: the distinct list is the exact distinct
    canonical set in first-occurrence order and queries return exact counts."""
    rs = synth.random_reads(31, 40, 30, 120, k=15, alphabet=b"ACG", p_n=0.01, p_other=0.01)
    reads = brute.split_reads(rs)
    exact = brute.exact_counts(reads, 15)
    X, Y = 2003, 2017
    keys = list(exact)
    slots = {(brute.h64(c) % X, brute.h64(c) % Y, brute.h64(c) % 8) for c in keys}
    assert len(slots) == len(keys), "seed gives a collision; pick another"
    bf = oracle_lib.CountBF(X, Y, 8, 1)
    distinct, nw = bf.insert(rs.reads, rs.offsets, 15)
    assert nw == sum(exact.values()) == sum(1 for _ in brute.windows(reads, 15))
    assert [int(x) for x in distinct] == keys
    q = bf.query(np.array(keys, dtype=np.uint64))
    assert [int(x) for x in q] == [min(v, 255) for v in exact.values()]
    assert int(bf.counters().sum()) == nw


def test_no_false_negatives_and_overcount(oracle_lib):
    """Every inserted k-mer queries >= min(exact count, 255) (Bloom-filter
    one-sided error), even in a heavily colliding filter."""
    rs = synth.random_reads(41, 50, 20, 80, k=11, alphabet=b"ACGT")
    reads = brute.split_reads(rs)
    exact = brute.exact_counts(reads, 11)
    bf = oracle_lib.CountBF(7, 11, 8, 2)
    bf.insert(rs.reads, rs.offsets, 11)
    q = bf.query(np.array(list(exact), dtype=np.uint64))
    for (k, v), got in zip(exact.items(), q):
        assert int(got) >= min(v, 255)


def test_saturation(oracle_lib):
    """A k-mer seen 300 times stops at 255 (reading of Algorithm 3's overflow
    check); no other counter changes."""
    K = 21
    rs = synth.reads_from_strings(["A" * (K + 299)], k=K)
    bf = oracle_lib.CountBF(101, 103, 8, 1)
    d, nw = bf.insert(rs.reads, rs.offsets, K)
    assert nw == 300 and len(d) == 1
    c = bf.counters()
    assert int(c.max()) == 255 and int(np.count_nonzero(c)) == 1
    bf5 = oracle_lib.CountBF(101, 103, 5, 1)
    bf5.insert(rs.reads, rs.offsets, K)
    assert int(bf5.counters().max()) == 31


def test_invalid_bases_skip_windows(oracle_lib):
    rs = synth.random_reads(51, 60, 5, 70, k=13, p_n=0.03, p_other=0.03)
    reads = brute.split_reads(rs)
    bf = oracle_lib.CountBF(97, 101, 8, 1)
    _, nw = bf.insert(rs.reads, rs.offsets, 13)
    assert nw == sum(1 for _ in brute.windows(reads, 13))


def test_strand_symmetry(oracle_lib):
    """Reads and their reverse complements give the same countBF (canonical
    k-mers, Sec. 2.3)."""
    rs = synth.random_reads(61, 70, 25, 100, k=17, p_n=0.01)
    reads = brute.split_reads(rs)
    rc = synth.reads_from_strings([brute.revcomp_str(s) for s in reads], k=17)
    a = oracle_lib.CountBF(61, 67, 8, 2)
    b = oracle_lib.CountBF(61, 67, 8, 2)
    da, _ = a.insert(rs.reads, rs.offsets, 17)
    db, _ = b.insert(rc.reads, rc.offsets, 17)
    assert np.array_equal(a.words, b.words)


def test_incremental_equals_concatenated(oracle_lib):
    a = synth.random_reads(71, 30, 20, 60, k=11)
    b = synth.random_reads(72, 40, 20, 60, k=11)
    ab = synth.concat_reads([a, b])
    one = oracle_lib.CountBF(23, 29, 8, 1)
    d1, _ = one.insert(ab.reads, ab.offsets, 11)
    two = oracle_lib.CountBF(23, 29, 8, 1)
    da, _ = two.insert(a.reads, a.offsets, 11)
    db, _ = two.insert(b.reads, b.offsets, 11)
    assert np.array_equal(one.words, two.words)
    assert np.array_equal(d1, np.concatenate([da, db]))


# --------------------------------------------------------------------------
# classification (Algorithm 2)
# --------------------------------------------------------------------------

def test_classify_partition_and_threshold(oracle_lib):
    rs = synth.random_reads(81, 200, 30, 120, k=9, alphabet=b"ACGT")
    reads = brute.split_reads(rs)
    exact = brute.exact_counts(reads, 9)
    bf = oracle_lib.CountBF(31, 37, 8, 1)
    distinct, _ = bf.insert(rs.reads, rs.offsets, 9)
    for tau in (0, 1, 2, 5, 254, 255):
        trust, err = bf.classify(distinct, tau)
        assert len(trust) + len(err) == len(distinct)
        q = bf.query(distinct)
        is_t = q > tau
        assert np.array_equal(trust, distinct[is_t])
        assert np.array_equal(err, distinct[~is_t])
        # one-sided error: truly trustworthy k-mers are never called erroneous
        errset = set(int(x) for x in err)
        for k, v in exact.items():
            if v > tau:
                assert k not in errset


def test_classify_exact_when_collision_free(oracle_lib):
    rs = synth.random_reads(91, 60, 40, 120, k=5, alphabet=b"ACGT")
    reads = brute.split_reads(rs)
    exact = brute.exact_counts(reads, 5)
    X, Y = 4001, 4003
    keys = list(exact)
    assert len({(brute.h64(c) % X, brute.h64(c) % Y, brute.h64(c) % 8) for c in keys}) == len(keys)
    bf = oracle_lib.CountBF(X, Y, 8, 1)
    distinct, _ = bf.insert(rs.reads, rs.offsets, 5)
    trust, err = bf.classify(distinct, 3)
    assert [int(x) for x in trust] == [k for k, v in exact.items() if min(v, 255) > 3]
    assert [int(x) for x in err] == [k for k, v in exact.items() if min(v, 255) <= 3]
