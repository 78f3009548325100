"""kc_insert_classify_noalloc (scratch in the library's fixed device array)
against kc_insert_classify on the same inputs, through the C ABI: two calls
in a row on one handle (the second with a smaller input, continuing the
countBF and the distinct list), every output equal, and both equal to the
oracle; inputs beyond the array's size are refused."""
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


def run(rs_list, X, Y, k, tau, noalloc):
    """Insert+classify each read set in turn into one handle; per call the
    (n_windows, distinct so far, trust, err) outputs, and the final words."""
    bf = P.CountBF(X, Y)
    total = sum(r.n_bases for r in rs_list)
    d = torch.empty(total, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    outs = []
    for rs in rs_list:
        r, o = dev(rs)
        t = torch.empty(rs.n_bases, dtype=torch.int64, device="cuda")
        e = torch.empty(rs.n_bases, dtype=torch.int64, device="cuda")
        args = dict(distinct=d, trust=t, err=e, n_distinct=cnt[0:1], n_windows=cnt[1:2],
                    n_trust=cnt[2:3], n_err=cnt[3:4])
        if noalloc:
            bf.insert_classify_noalloc(r, o, k, tau, **args)
        else:
            bf.insert_classify(r, o, k, tau, **args)
        bf.sync()
        nd, nw, nt, ne = (int(x) for x in cnt.cpu())
        outs.append((nw, d[:nd].cpu().numpy().view(np.uint64).copy(),
                     t[:nt].cpu().numpy().view(np.uint64).copy(),
                     e[:ne].cpu().numpy().view(np.uint64).copy()))
    words = bf.words.cpu().numpy().view(np.uint64).copy()
    bf.close()
    return outs, words


@pytest.mark.parametrize("X,Y", [(269, 281), (1201, 1213)])
def test_noalloc_equals_insert_classify_twice(X, Y):
    a = synth.config("tiny", 1.0)             # 1 M bases
    b = synth.random_reads(2500, 2000, 60, 200, k=21, p_n=0.01)  # a smaller second call
    assert b.n_bases < a.n_bases
    print(f"case noalloc X={X} Y={Y} calls of {a.n_bases} then {b.n_bases} bases", flush=True)
    ref, ref_words = run([a, b], X, Y, 21, 2, noalloc=False)
    got, got_words = run([a, b], X, Y, 21, 2, noalloc=True)
    assert np.array_equal(got_words, ref_words)
    for (gw, gd, gt, ge), (rw, rd, rt, re) in zip(got, ref):
        assert gw == rw
        assert np.array_equal(gd, rd) and np.array_equal(gt, rt) and np.array_equal(ge, re)
    # and the oracle: the same two inserts, each call's split of its new keys
    bf = oracle.CountBF(X, Y)
    d1, w1 = bf.insert(a.reads, a.offsets, 21)
    t1, e1 = bf.classify(d1, 2)
    assert got[0][0] == w1 and np.array_equal(got[0][1], d1)
    assert np.array_equal(got[0][2], t1) and np.array_equal(got[0][3], e1)
    d2, w2 = bf.insert(b.reads, b.offsets, 21)
    t2, e2 = bf.classify(d2, 2)
    # the window counter accumulates over calls; the list continues
    assert got[1][0] == w1 + w2 and np.array_equal(got[1][1], np.concatenate([d1, d2]))
    assert np.array_equal(got[1][2], t2) and np.array_equal(got[1][3], e2)
    assert np.array_equal(got_words, bf.words)


def test_noalloc_refuses_what_does_not_fit():
    rs = synth.random_reads(2600, 40_000, 100, 100, k=21)  # 4 M bases: beyond the array
    X, Y = 269, 281
    assert P.scratch_bytes(X, Y, rs.n_bases) > (64 << 20)
    bf = P.CountBF(X, Y)
    r, o = dev(rs)
    z = [torch.zeros(max(1, rs.n_bases), dtype=torch.int64, device="cuda") for _ in range(3)]
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(P.KmercoError) as ex:
        bf.insert_classify_noalloc(r, o, 21, 2, z[0], z[1], z[2], c[0:1], c[1:2], c[2:3], c[3:4])
    assert ex.value.status == P.KC_ERANGE
    bf.sync()
    assert int(c.abs().sum()) == 0 and not bool(bf.words.any())  # nothing was enqueued
    bf.close()


def test_noalloc_in_several_chunks(monkeypatch):
    """An insert of several chunks (chunk size forced small) through the
    allocation-free entry point: its carried first-seen records are carved
    from the fixed array too; equal to kc_insert_classify and the oracle."""
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "131072")
    a = synth.config("tiny", 1.0)
    X, Y = 269, 281
    bf = P.CountBF(X, Y)
    plan = bf.plan(a.n_bases)
    bf.close()
    assert plan["n_chunks"] > 2 and plan["carried"] == 1, plan
    print(f"case noalloc in {plan['n_chunks']} chunks", flush=True)
    ref, ref_words = run([a], X, Y, 21, 2, noalloc=False)
    got, got_words = run([a], X, Y, 21, 2, noalloc=True)
    assert np.array_equal(got_words, ref_words)
    (gw, gd, gt, ge), (rw, rd, rt, re) = got[0], ref[0]
    assert gw == rw and np.array_equal(gd, rd)
    assert np.array_equal(gt, rt) and np.array_equal(ge, re)
    words, d, t, e, nw = oracle.run_kmerco(a.reads, a.offsets, 21, 2, X, Y)
    assert np.array_equal(got_words, words) and gw == nw
    assert np.array_equal(gd, d) and np.array_equal(gt, t) and np.array_equal(ge, e)
