"""Checkpoint / resume of a countBF (``CountBF.save`` / ``CountBF.load``):
inserting A, saving, loading in a new handle and inserting B gives the
oracle's result for A followed by B (incremental insertion: several calls
equal one call on the concatenated reads)."""
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


@pytest.mark.parametrize("k,alpha,k_h", [(25, 8, 1), (21, 4, 2), (40, 8, 1)])
def test_save_load_continues_the_filter(tmp_path, k, alpha, k_h):
    a = synth.random_reads(1700 + k, 700, 40, 200, k=k, p_n=0.01, alphabet=b"ACG")
    b = synth.random_reads(1800 + k, 900, 40, 200, k=k, p_n=0.01, alphabet=b"ACG")
    ab = synth.concat_reads([a, b])
    X, Y = 211, 223
    print(f"case checkpoint k={k} alpha={alpha} k_h={k_h}", flush=True)
    words, distinct, _, _, _ = oracle.run_kmerco(ab.reads, ab.offsets, k, 2, X, Y, alpha, k_h)
    w = P.key_words(k)

    bf = P.CountBF(X, Y, alpha, k_h)
    ra, oa = dev(a)
    d = bf.insert(ra, oa, k)
    path = tmp_path / "countbf.npz"
    bf.save(path, distinct=d)
    bf.close()

    bf2, saved = P.CountBF.load(path)
    assert bf2.k == k and (bf2.layout.X, bf2.layout.Y) == (X, Y)
    assert (bf2.layout.alpha, bf2.layout.k_h) == (alpha, k_h)
    out = torch.empty(ab.n_bases * w, dtype=torch.int64, device="cuda")
    out[:saved.numel()] = saved
    rb, ob = dev(b)
    bf2.insert(rb, ob, k, distinct=out)
    bf2.sync()
    n = int(bf2.n_distinct.item())
    got = out[:n * w].cpu().numpy().view(np.uint64)
    assert np.array_equal(bf2.words.cpu().numpy().view(np.uint64),
                          np.asarray(words, dtype=np.uint64))
    assert np.array_equal(got, np.asarray(distinct, dtype=np.uint64).reshape(-1))
    bf2.close()


def test_load_without_distinct(tmp_path):
    rs = synth.random_reads(1900, 300, 40, 120, k=21)
    bf = P.CountBF(101, 103)
    r, o = dev(rs)
    bf.insert(r, o, 21)
    path = tmp_path / "words_only.npz"
    bf.save(path)
    bf2, saved = P.CountBF.load(path)
    assert saved is None and int(bf2.n_distinct.item()) == 0
    assert torch.equal(bf2.words, bf.words)
    with np.load(path, allow_pickle=False) as z:  # plain arrays only
        assert sorted(z.files) == ["layout", "words"]


@pytest.mark.parametrize("k", [40, 25])
def test_load_then_classify_and_query_before_any_insert(tmp_path, k):
    """A resumed handle carries the saved k: classify and query read keys of
    that width before any insert (two words per key for k > 32)."""
    rs = synth.random_reads(2000 + k, 600, 50, 160, k=k, p_n=0.01, alphabet=b"ACG")
    X, Y, tau = 199, 211, 2
    print(f"case load-then-classify k={k}", flush=True)
    ref = oracle.CountBF(X, Y)
    distinct, _ = ref.insert(rs.reads, rs.offsets, k)
    trust, err = ref.classify(distinct, tau)
    freq = ref.query(distinct)
    w = P.key_words(k)

    bf = P.CountBF(X, Y)
    r, o = dev(rs)
    d = bf.insert(r, o, k)
    path = tmp_path / "resume.npz"
    bf.save(path, distinct=d)
    bf.close()

    bf2, saved = P.CountBF.load(path)
    n = saved.numel() // w
    t, nt, e, ne = bf2.classify(saved, torch.tensor([n], dtype=torch.int64, device="cuda"), tau)
    f = bf2.query(saved)
    bf2.sync()
    u = lambda x, m: x[:m * w].cpu().numpy().view(np.uint64)  # noqa: E731
    assert np.array_equal(u(t, int(nt.item())), np.asarray(trust, dtype=np.uint64).reshape(-1))
    assert np.array_equal(u(e, int(ne.item())), np.asarray(err, dtype=np.uint64).reshape(-1))
    assert np.array_equal(f.cpu().numpy().astype(np.uint64), np.asarray(freq, dtype=np.uint64))
    # a resumed handle refuses inserts of another k
    with pytest.raises(P.KmercoError) as ex:
        bf2.insert(r, o, k + 1)
    assert ex.value.status == P.KC_ESTATE
    bf2.close()


def test_rejected_insert_does_not_set_k():
    """An insert refused by the checks (a k above 32 on the direct path) leaves
    the handle without a k, so a later valid insert of another k runs."""
    import os
    rs = synth.random_reads(2100, 200, 50, 120, k=21)
    r, o = dev(rs)
    os.environ["KMERCO_PATH"] = "direct"
    try:
        bf = P.CountBF(101, 103)  # the direct path takes k <= 32 only
    finally:
        del os.environ["KMERCO_PATH"]
    with pytest.raises(P.KmercoError) as ex:
        bf.insert(r, o, 40)
    assert ex.value.status == P.KC_EINVAL
    bf.insert(r, o, 21)
    bf.sync()
    words, distinct, _, _, _ = oracle.run_kmerco(rs.reads, rs.offsets, 21, 2, 101, 103)
    assert np.array_equal(bf.words.cpu().numpy().view(np.uint64), words)
    assert int(bf.n_distinct.item()) == len(distinct)
    bf.close()
