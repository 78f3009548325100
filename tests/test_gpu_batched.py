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
            room = (nb + extra + 64) * P.key_words(rs.k)  # distinct <= windows <= bases
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
            w = P.key_words(e["k"])
            lst = lambda t, n: u(t[:n * w]).reshape(-1, 2) if w == 2 else u(t[:n])  # noqa: E731
            nd = int(e["n_distinct"].item())
            r = {"words": u(e["filter"].words), "distinct": lst(e["distinct"], nd),
                 "nw": int(e["n_windows"].item())}
            if "trust" in e:
                r["trust"] = lst(e["trust"], int(e["n_trust"].item()))
                r["err"] = lst(e["err"], int(e["n_err"].item()))
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
    wide = [dict(e) for e in run.entries]
    wide[0]["k"] = 65  # beyond the longest k-mer
    with pytest.raises(P.KmercoError):
        b.insert(wide, run.reads, run.offs)
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


def side_lane_cases():
    """Sets the fused phase kernels do not take, mixed with ones they do: a
    countBF of 8229 regions (single-level binned, beyond the fused form's
    2048), one of 16,448 regions (the partitioned path), 40-mers (two-word
    keys), an empty set, and small sets around them."""
    small = mixed_cases(7)
    big_reads = synth.random_reads(8100, 9000, 80, 250, k=31, tau=3, p_n=0.002)
    part_reads = synth.random_reads(8200, 6000, 60, 200, k=27, tau=2, p_n=0.002)
    wide_reads = synth.random_reads(8300, 3000, 50, 220, k=40, tau=2, p_n=0.002,
                                    alphabet=b"ACGT")
    empty = synth.reads_from_strings([], k=21, tau=2)
    return [small[0], (big_reads, (4099, 4111, 8, 1), True), small[1],
            (part_reads, (5801, 5807, 8, 1), True), (wide_reads, (307, 311, 8, 1), True),
            small[2], (empty, (101, 103, 8, 1), True), small[3]]


def test_side_lane_sets_eager_graph_and_tuned():
    """Every set equals the oracle run on it alone: eager, then captured and
    replayed three times with unrelated eager work between the replays, then
    with the tuner (work-item size and the side sets' chunk sizes)."""
    cases = side_lane_cases()
    want = oracle_each(cases)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        run = BatchRun(cases, stream=stream)
        b = P.Batch()
        print("case side lanes: eager", flush=True)
        b.insert(run.entries, run.reads, run.offs, reset=True, stream=stream)
        assert_sets_equal(run.results(), want, "side lanes eager")
        for rep in range(3):
            print(f"case side lanes: graph replay {rep}", flush=True)
            b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
            assert_sets_equal(run.results(), want, f"side lanes graph {rep}")
            x = torch.arange(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            assert int(x.item()) == (1 << 20) * ((1 << 20) - 1) // 2
        print("case side lanes: tuned", flush=True)
        b.insert(run.entries, run.reads, run.offs, reset=True, tune=True, stream=stream)
        assert_sets_equal(run.results(), want, "side lanes tuned")
        b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
        assert_sets_equal(run.results(), want, "side lanes tuned, graph")


def test_side_lane_full_chunk_partitioned_digests():
    """A set of 280 M bases (more than one 2^28-base chunk of the fused form)
    into a 269 MB countBF (16,448 regions: the partitioned path) between two
    small sets, tuned and graph-captured, against the oracle's digests of
    that input and the oracle on the small sets."""
    import hashlib
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "fullchunk_5801x5807_digests.json")))
    rs = synth.random_reads(1500, 1_400_000, 150, 250, k=31, p_n=0.0005, tau=3)
    assert rs.n_bases == ref["n_bases"] and rs.n_bases > (1 << 28)
    small = mixed_cases(8)
    cases = [small[0], (rs, (5801, 5807, 8, 1), True), small[1]]
    print(f"case side lane full chunk partitioned: {rs.n_bases} bases", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        run = BatchRun(cases, stream=stream)
        b = P.Batch()
        b.insert(run.entries, run.reads, run.offs, reset=True, tune=True, stream=stream)
        b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
        got = run.results()

    def h(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()

    g = got[1]
    assert g["nw"] == ref["n_windows"]
    assert (len(g["distinct"]), len(g["trust"]), len(g["err"])) == \
        (ref["n_distinct"], ref["n_trust"], ref["n_err"])
    assert h(g["words"]) == ref["words_sha256"] and h(g["distinct"]) == ref["distinct_sha256"]
    assert h(g["trust"]) == ref["trust_sha256"] and h(g["err"]) == ref["err_sha256"]
    want = oracle_each([small[0], small[1]])
    assert_sets_equal([got[0], got[2]], want, "small sets beside the large one")


def test_side_lane_sets_in_several_chunks(monkeypatch):
    """Side-lane sets inserted in several chunks (chunk size forced small):
    their split takes the carried classification (the last chunk's region
    pass marks the earlier chunks' first-seen k-mers from records kept in the
    side lane's workspace), eager and graph-replayed, equal to the oracle."""
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "65536")
    cases = side_lane_cases()
    want = oracle_each(cases)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        run = BatchRun(cases, stream=stream)
        plans = [e["filter"].plan(e["n_bases"]) for e in run.entries]
        assert any(p["n_chunks"] > 1 and p["carried"] for p in plans), plans
        b = P.Batch()
        print("case side lanes in chunks: eager", flush=True)
        b.insert(run.entries, run.reads, run.offs, reset=True, stream=stream)
        assert_sets_equal(run.results(), want, "side lanes in chunks, eager")
        for rep in range(2):
            print(f"case side lanes in chunks: graph replay {rep}", flush=True)
            b.insert(run.entries, run.reads, run.offs, reset=True, graph=True, stream=stream)
            assert_sets_equal(run.results(), want, f"side lanes in chunks, graph {rep}")
