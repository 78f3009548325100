"""Handles whose device state lives in caller memory (kc_create_in with a
scratch buffer): inserts allocate nothing and never wait on the host, so a
caller can capture them in a HIP graph; every replay equals the oracle."""
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


def u64(t, n):
    return t[:n].cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("X,Y,part_log", [(269, 281, None), (601, 607, 2)])
def test_caller_scratch_insert_under_graph_capture(monkeypatch, X, Y, part_log):
    """kc_reset + kc_insert_classify on a caller-scratch handle, captured once
    and replayed four times with unrelated eager work in between; each
    replay's countBF, distinct list and split equal the oracle's.  The second
    case forces the partitioned path (partitions of 4 regions)."""
    if part_log is not None:
        monkeypatch.setenv("KMERCO_PART_LOG", str(part_log))
    rs = synth.config("tiny", 0.3)
    print(f"case graph-capture caller scratch X={X} Y={Y} part_log={part_log}", flush=True)
    words, distinct, trust, err, nw = oracle.run_kmerco(rs.reads, rs.offsets, rs.k, rs.tau, X, Y)
    need = P.scratch_bytes(X, Y, rs.n_bases)
    assert need % 256 == 0
    scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
    bf = P.CountBF(X, Y, scratch=scratch, max_bases=rs.n_bases)
    r, o = dev(rs)
    cap = rs.n_bases
    out = {n: torch.empty(cap, dtype=torch.int64, device="cuda") for n in ("d", "t", "e")}
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()

    def step():
        bf.reset(stream=s)
        cnt.zero_()
        bf.insert_classify(r, o, rs.k, rs.tau, distinct=out["d"], trust=out["t"], err=out["e"],
                           n_distinct=cnt[0:1], n_windows=cnt[1:2], n_trust=cnt[2:3],
                           n_err=cnt[3:4], stream=s)

    def check():
        nd, n_w, nt, ne = (int(x) for x in cnt.cpu())
        assert n_w == nw
        assert np.array_equal(bf.words.cpu().numpy().view(np.uint64), words)
        assert np.array_equal(u64(out["d"], nd), distinct)
        assert np.array_equal(u64(out["t"], nt), trust)
        assert np.array_equal(u64(out["e"], ne), err)

    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # eager, outside the graph
    s.synchronize()
    bf.sync()
    check()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    noise = torch.arange(1 << 20, device="cuda")
    for rep in range(4):
        out["d"].fill_(-1)
        noise.mul_(3).add_(rep)  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check()
    del g
    bf.close()


def test_caller_scratch_limits():
    """Too little scratch fails at creation; an insert larger than max_bases
    or a misaligned buffer is refused; smaller inserts still run."""
    rs = synth.config("tiny", 0.2)
    X, Y = 269, 281
    need = P.scratch_bytes(X, Y, rs.n_bases)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.KmercoError) as ex:
        P.CountBF(X, Y, scratch=small, max_bases=rs.n_bases)
    assert ex.value.status == P.KC_ERANGE
    buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.KmercoError) as ex:
        P.CountBF(X, Y, scratch=buf[1:], max_bases=rs.n_bases)
    assert ex.value.status == P.KC_EINVAL
    half = rs.n_reads // 2
    bf = P.CountBF(X, Y, scratch=buf[:need], max_bases=int(rs.offsets[half]))
    r, o = dev(rs)
    with pytest.raises(P.KmercoError) as ex:
        bf.insert(r, o, rs.k)
    assert ex.value.status == P.KC_ERANGE
    a = rs.subset(0, half)
    ra, oa = dev(a)
    bf.insert(ra, oa, rs.k)
    bf.sync()
    words, distinct, _, _, _ = oracle.run_kmerco(a.reads, a.offsets, rs.k, rs.tau, X, Y)
    assert np.array_equal(bf.words.cpu().numpy().view(np.uint64), words)
    assert int(bf.n_distinct.item()) == len(distinct)
    bf.close()
