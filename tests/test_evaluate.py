"""The evaluation's exact counting (plain numpy) against brute force from the
definitions, its reverse complement against the paper's worked example, and
its comparison of KmerCo lists with exact counts on the oracle's outputs
(whose properties are fixed: reported k-mers exist, trustworthy + erroneous
partition the distinct list, counters never under-count)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2305_07545_amd import evaluate as E
from tests import brute


@pytest.mark.parametrize("k", [1, 2, 7, 13, 31, 32])
def test_exact_counts_match_brute_force(k):
    rs = synth.random_reads(40 + k, 150, 1, 120, k=k, tau=2, p_n=0.02, p_other=0.01)
    keys, cnt = E.exact_counts(rs.reads, rs.offsets, k)
    ref = brute.exact_counts(brute.split_reads(rs), k)
    rk = E.strand_free(np.array(list(ref.keys()), dtype=np.uint64), k)
    order = np.argsort(rk)
    assert np.array_equal(rk[order], keys)
    assert np.array_equal(np.array(list(ref.values()), dtype=np.int64)[order], cnt)
    assert cnt.sum() == sum(1 for _ in brute.windows(brute.split_reads(rs), k))


def test_revcomp_keys():
    rng = np.random.default_rng(3)
    for k in (1, 5, 28, 31, 32):
        strs = ["".join(rng.choice(list("ACGT"), size=k)) for _ in range(50)]
        keys = np.array([brute.key_of(s) for s in strs], dtype=np.uint64)
        want = np.array([brute.key_of(brute.revcomp_str(s)) for s in strs], dtype=np.uint64)
        assert np.array_equal(E.revcomp_keys(keys, k), want)
    # the paper's example (Sec. 2.2): the reverse complement of ATTGCGA is TCGCAAT
    assert E.revcomp_keys(np.array([brute.key_of("ATTGCGA")], dtype=np.uint64), 7)[0] == \
        brute.key_of("TCGCAAT")


@pytest.mark.parametrize("XY", [(3, 5), (61, 67), (2003, 2011)])
def test_compare_on_oracle_outputs(XY):
    """Small filters collide (missed distinct k-mers, over-counts); a large
    one is nearly exact.  The fixed properties hold at every size."""
    oracle.build(force=False)
    rs = synth.config("tiny", scale=0.2)  # 10x coverage: repeated k-mers
    k, tau = rs.k, rs.tau
    words, distinct, trust, err, nw = oracle.run_kmerco(rs.reads, rs.offsets, k, tau, *XY)
    keys, cnt = E.exact_counts(rs.reads, rs.offsets, k)
    r = E.compare(keys, cnt, distinct, trust, err, k, tau)
    assert r["exact_trustworthy"] > 1000
    assert r["distinct_unique"] and r["distinct_all_exist"] and r["split_is_partition"]
    assert r["trustworthy_missed_among_reported"] == 0
    assert int(cnt.sum()) == nw
    assert r["trustworthy_recall"] <= 1.0 and r["distinct_recall"] <= 1.0
    if XY == (2003, 2011):
        assert r["distinct_recall"] > 0.95 and r["trustworthy_precision"] > 0.95
    if XY == (3, 5):
        assert r["distinct_recall"] < 0.01


def test_placement():
    assert E.placement(491_000) == "L2 (one XCD)"
    assert E.placement(55_711_976) == "Infinity Cache"
    assert E.placement(8_013_000_000) == "HBM"
