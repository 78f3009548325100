"""k-mers of 33..64 bases (128-bit keys) through the HIP path, bit-exact
against the oracle: countBF words, distinct / trustworthy / erroneous lists
as (low, high) word pairs, window counts; fused and separate
classification, several hash functions, many chunks, the partitioned path,
Query-II; and the calls that do not take such keys."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2305_07545_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    P.load_library()


def dev(rs):
    return (torch.from_numpy(rs.reads).cuda(),
            torch.from_numpy(rs.offsets.view(np.int64)).cuda())


def check(rs, k, tau, X, Y, alpha=8, k_h=1, fused=True, what=""):
    print(f"case wide {what}: k={k} X={X} Y={Y} alpha={alpha} k_h={k_h} fused={fused} "
          f"bases={rs.n_bases}", flush=True)
    g = P.run_kmerco(*dev(rs), k, tau, X, Y, alpha, k_h, fused=fused)
    c = oracle.run_kmerco(rs.reads, rs.offsets, k, tau, X, Y, alpha, k_h)
    for name, a, b in zip(["words", "distinct", "trust", "err"], g[:4], c[:4]):
        a = np.asarray(a, dtype=np.uint64)
        b = np.asarray(b, dtype=np.uint64)
        assert a.shape == b.shape, f"{what} {name}: {a.shape} != {b.shape}"
        assert np.array_equal(a, b), f"{what} {name}: {int((a != b).sum())} mismatches"
    assert g[4] == c[4]
    return g


@pytest.mark.parametrize("k", [33, 45, 55, 64])
def test_wide_keys_match_oracle(k):
    rs = synth.random_reads(900 + k, 1500, 1, 400, k=k, tau=2, p_n=0.01, p_other=0.005)
    for X, Y in [(3, 5), (257, 263), (2003, 2011)]:
        check(rs, k, 2, X, Y, what=f"k={k}")
    check(rs, k, 2, 257, 263, fused=False, what=f"k={k} unfused")


@pytest.mark.parametrize("alpha,k_h", [(8, 2), (5, 3), (16, 1)])
def test_wide_layouts_and_hash_functions(alpha, k_h):
    rs = synth.random_reads(950 + alpha + k_h, 1000, 60, 300, k=55, tau=3, p_n=0.01)
    check(rs, 55, 3, 211, 223, alpha, k_h, what=f"a={alpha} kh={k_h}")


def test_wide_repeats_saturate():
    """A genome sampled at high coverage: repeated 55-mers, saturating
    counters at alpha = 4, trustworthy ones."""
    rs = synth.config("tiny", scale=0.3)
    check(rs, 55, 3, 101, 103, alpha=4, what="tiny 55-mers, alpha 4")
    check(rs, 40, 3, 1009, 1013, what="tiny 40-mers")


def test_wide_multi_chunk_and_partitions(monkeypatch):
    rs = synth.random_reads(980, 800, 30, 300, k=51, tau=2, p_n=0.01)
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "4096")
    check(rs, 51, 2, 257, 263, what="chunks of 4096")
    monkeypatch.delenv("KMERCO_CHUNK_POSITIONS")
    monkeypatch.setenv("KMERCO_PATH", "binned")
    monkeypatch.setenv("KMERCO_PART_LOG", "2")
    check(rs, 51, 2, 257, 263, what="partitions of 4 regions")
    check(rs, 51, 2, 257, 263, k_h=2, what="partitions of 4 regions, k_h 2")


def test_wide_query_and_classify_calls():
    rs = synth.random_reads(990, 500, 80, 200, k=60, tau=2, p_n=0.01)
    X, Y = 211, 223
    reads, offs = dev(rs)
    bf = P.CountBF(X, Y, 8, 2)
    distinct = bf.insert(reads, offs, 60)
    bf.sync()
    nd = int(bf.n_distinct.item())
    ob = oracle.CountBF(X, Y, 8, 2)
    od, _ = ob.insert(rs.reads, rs.offsets, 60)
    keys = distinct[:2 * nd]
    assert np.array_equal(keys.cpu().numpy().view(np.uint64).reshape(-1, 2), od)
    freq = bf.query(keys).cpu().numpy()
    assert np.array_equal(freq.astype(np.uint64), ob.query(od))
    trust, n_trust, err, n_err = bf.classify(keys, bf.n_distinct, 2)
    bf.sync()
    ot, oe = ob.classify(od, 2)
    t = trust[:2 * int(n_trust.item())].cpu().numpy().view(np.uint64).reshape(-1, 2)
    e = err[:2 * int(n_err.item())].cpu().numpy().view(np.uint64).reshape(-1, 2)
    assert np.array_equal(t, ot) and np.array_equal(e, oe)


def test_wide_keys_rejected_where_unsupported(monkeypatch):
    rs = synth.random_reads(995, 20, 60, 100, k=40)
    reads, offs = dev(rs)
    monkeypatch.setenv("KMERCO_PATH", "direct")
    bf = P.CountBF(101, 103)
    with pytest.raises(P.KmercoError):
        bf.insert(reads, offs, 40)
    monkeypatch.delenv("KMERCO_PATH")
    with pytest.raises(P.KmercoError):
        P.CountBF(101, 103).insert(reads, offs, 65)
