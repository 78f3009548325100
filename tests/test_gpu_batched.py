"""Batched form: every set's outputs must equal the oracle run on that set
alone (bit-exact), in eager mode, under HIP-graph capture and replay, and
with the work-item size autotuned."""
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


def u(t):
    return t.cpu().numpy().view(np.uint64)


class BatchRun:
    """Filters, outputs and packed reads for a list of
    (ReadSet, (X, Y, alpha, k_h), split) cases."""

    def __init__(self, cases, stream=None, extra=0):
        self.cases = cases
        self.stream = stream
        reads, offs, self.spans = P.pack_read_sets([(rs.reads, rs.offsets) for rs, _, _ in cases])
        self.reads = torch.from_numpy(reads).cuda()
        self.offs = torch.from_numpy(offs.view(np.int64)).cuda()
        self.entries = []
        for (rs, (X, Y, a, kh), split), (base, nb, _, _) in zip(cases, self.spans):
            f = P.CountBF(X, Y, a, kh, stream=stream)
            room = nb + extra + 64  # distinct <= windows <= bases
            e = {"filter": f, "first_base": base, "n_bases": nb, "k": rs.k, "tau": rs.tau,
                 "distinct": torch.empty(room, dtype=torch.int64, device="cuda"),
                 "n_distinct": torch.zeros(1, dtype=torch.int64, device="cuda"),
                 "n_windows": torch.zeros(1, dtype=torch.int64, device="cuda")}
            if split:
                e.update({"trust": torch.empty(room, dtype=torch.int64, device="cuda"),
                          "err": torch.empty(room, dtype=torch.int64, device="cuda"),
                          "n_trust": torch.zeros(1, dtype=torch.int64, device="cuda"),
                          "n_err": torch.zeros(1, dtype=torch.int64, device="cuda")})
            self.entries.append(e)

    def results(self):
        torch.cuda.synchronize()
        out = []
        for e in self.entries:
            e["filter"].sync()
            nd = int(e["n_distinct"].item())
            r = {"words": u(e["filter"].words), "distinct": u(e["distinct"][:nd]),
                 "nw": int(e["n_windows"].item())}
            if "trust" in e:
                r["trust"] = u(e["trust"][:int(e["n_trust"].item())])
                r["err"] = u(e["err"][:int(e["n_err"].item())])
            out.append(r)
        return out


def oracle_each(cases):
    out = []
    for rs, (X, Y, a, kh), split in cases:
        w, d, t, e, nw = oracle.run_kmerco(rs.reads, rs.offsets, rs.k, rs.tau, X, Y, a, kh)
        out.append({"words": w, "distinct": d, "trust": t, "err": e, "nw": nw, "split": split})
    return out


def assert_sets_equal(got, want, what=""):
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g["words"], w["words"]), f"{what} set {i}: words"
        assert np.array_equal(g["distinct"], w["distinct"]), f"{what} set {i}: distinct"
        assert g["nw"] == w["nw"], f"{what} set {i}: windows {g['nw']} != {w['nw']}"
        if w["split"]:
            assert np.array_equal(g["trust"], w["trust"]), f"{what} set {i}: trust"
            assert np.array_equal(g["err"], w["err"]), f"{what} set {i}: err"


def mixed_cases(seed=0):
    rng = np.random.default_rng(seed)
    layouts = [(31, 37, 8, 1), (101, 103, 8, 1), (211, 223, 8, 2), (503, 509, 8, 1),
               (97, 101, 5, 1), (61, 67, 16, 3), (13, 17, 8, 1), (401, 409, 12, 1)]
    cases = []
    for i in range(12):
        k = int(rng.choice([9, 13, 21, 25, 31, 32]))
        n = 0 if i == 5 else int(rng.integers(1, 1500))
        rs = synth.random_reads(5000 + seed * 100 + i, max(n, 1), 20, 300, k=k,
                                tau=int(rng.integers(0, 6)), p_n=0.005)
        if n == 0:
            rs = synth.reads_from_strings([], k=k, tau=2)
        cases.append((rs, layouts[i % len(layouts)], i % 4 != 3))
    return cases


def test_mixed_sets_eager():
    cases = mixed_cases(0)
    print("case mixed eager: sets", len(cases), flush=True)
    run = BatchRun(cases)
    b = P.Batch()
    b.insert(run.entries, run.reads, run.offs, reset=True)
    assert_sets_equal(run.results(), oracle_each(cases), "eager")


def test_graph_replays_match_eager():
    """Capture once, replay several times with eager work and syncs between
    the replays; every replay must reproduce the oracle's outputs."""
    cases = mixed_cases(1)
    want = oracle_each(cases)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        run = BatchRun(cases, stream=stream)
        b = P.Batch()
        for rep in range(4):
            print(f"case graph replay {rep}", flush=True)
            b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
            assert_sets_equal(run.results(), want, f"graph replay {rep}")
            # unrelated eager work on the same device between replays
            x = torch.arange(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            assert int(x.item()) == (1 << 20) * ((1 << 20) - 1) // 2


def test_autotune_keeps_results():
    cases = mixed_cases(2)
    run = BatchRun(cases)
    b = P.Batch()
    print("case autotune", flush=True)
    b.insert(run.entries, run.reads, run.offs, reset=True, tune=True)
    assert b.tile in (16384, 32768, 65536, 131072, 262144)
    assert_sets_equal(run.results(), oracle_each(cases), "tuned")
    b.tile = 16384
    b.insert(run.entries, run.reads, run.offs, reset=True)
    assert_sets_equal(run.results(), oracle_each(cases), "tile 16384")


def test_incremental_batches():
    a = mixed_cases(3)
    bb = [(synth.random_reads(7000 + i, 300, 20, 200, k=rs.k, tau=rs.tau), lay, split)
          for i, (rs, lay, split) in enumerate(a)]
    # insert-only so that distinct lists concatenate across the two calls
    a = [(rs, lay, False) for rs, lay, _ in a]
    bb = [(rs, lay, False) for rs, lay, _ in bb]
    # the second call brings at most 300 * 200 more windows per set
    run_a = BatchRun(a, extra=300 * 200)
    batch = P.Batch()
    batch.insert(run_a.entries, run_a.reads, run_a.offs, reset=True)
    reads_b, offs_b, spans_b = P.pack_read_sets([(rs.reads, rs.offsets) for rs, _, _ in bb])
    entries_b = []
    for e, (base, nb, _, _) in zip(run_a.entries, spans_b):
        e2 = dict(e)
        e2["first_base"], e2["n_bases"] = base, nb
        entries_b.append(e2)
    print("case incremental batches", flush=True)
    batch.insert(entries_b, torch.from_numpy(reads_b).cuda(),
                 torch.from_numpy(offs_b.view(np.int64)).cuda())
    got = run_a.results()
    for i, ((rs1, lay, _), (rs2, _, _)) in enumerate(zip(a, bb)):
        both = synth.concat_reads([rs1, rs2])
        w, d, _, _, nw = oracle.run_kmerco(both.reads, both.offsets, rs1.k, rs1.tau, *lay)
        assert np.array_equal(got[i]["words"], w), f"set {i} words"
        assert np.array_equal(got[i]["distinct"], d), f"set {i} distinct"
        assert got[i]["nw"] == nw


def test_batched_workload_small_scale():
    sets = synth.config("batched", scale=0.004)
    cases = []
    for rs in sets:
        X, Y = oracle.dims(rs.n_items)
        cases.append((rs, (X, Y, 8, 1), True))
    print(f"case batched workload x0.004: {len(cases)} sets", flush=True)
    run = BatchRun(cases)
    b = P.Batch()
    b.insert(run.entries, run.reads, run.offs, reset=True, tune=True)
    assert_sets_equal(run.results(), oracle_each(cases), "batched workload")


def test_batch_argument_errors():
    cases = mixed_cases(4)[:3]
    run = BatchRun(cases)
    b = P.Batch()
    bad = [dict(e) for e in run.entries]
    bad[1]["first_base"] += 1  # misaligned set
    with pytest.raises(P.KmercoError):
        b.insert(bad, run.reads, run.offs)
    dup = [dict(e) for e in run.entries]
    dup[2]["filter"] = dup[0]["filter"]  # one filter for two sets
    with pytest.raises(P.KmercoError):
        b.insert(dup, run.reads, run.offs)
    big = [dict(e) for e in run.entries]
    big[0]["filter"] = P.CountBF(4099, 4111)  # 2^14 regions: beyond the batched limit
    with pytest.raises(P.KmercoError):
        b.insert(big, run.reads, run.offs)
    with pytest.raises(P.KmercoError):
        b.insert(run.entries, run.reads, run.offs, graph=True, stream=torch.cuda.default_stream())


def test_batched_workload_full_size_digests():
    """All 256 sets of the batched workload at full size in one graph-captured
    batched call, against the oracle's per-set digests."""
    import hashlib
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "batched_digests.json")))["sets"]
    sets = synth.config("batched")
    cases = [(rs, (r["X"], r["Y"], 8, 1), True) for rs, r in zip(sets, ref)]
    print(f"case batched workload full size: {len(cases)} sets", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        run = BatchRun(cases, stream=stream)
        b = P.Batch()
        b.insert(run.entries, run.reads, run.offs, reset=True, tune=True, stream=stream)
        b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
        got = run.results()

    def h(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()

    for i, (g, r) in enumerate(zip(got, ref)):
        assert g["nw"] == r["n_windows"], f"set {i} windows"
        assert len(g["distinct"]) == r["n_distinct"], f"set {i} distinct count"
        assert h(g["words"]) == r["words_sha256"], f"set {i} words"
        assert h(g["distinct"]) == r["distinct_sha256"], f"set {i} distinct"
        assert h(g["trust"]) == r["trust_sha256"], f"set {i} trust"
        assert h(g["err"]) == r["err_sha256"], f"set {i} err"
