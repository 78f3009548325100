"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every GPU output -- countBF words, distinct list (order included),
trustworthy / erroneous lists and the inserted-window count -- must equal
the oracle's exactly: all outputs are integers and the readings taken make
each of them unique."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2305_07545_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    P.load_library()


def dev(rs):
    reads = torch.from_numpy(rs.reads).cuda()
    offs = torch.from_numpy(rs.offsets.view(np.int64)).cuda()
    return reads, offs


def gpu_run(rs, X, Y, alpha=8, k_h=1, k=None, tau=None, fused=True):
    reads, offs = dev(rs)
    return P.run_kmerco(reads, offs, rs.k if k is None else k, rs.tau if tau is None else tau,
                        X, Y, alpha, k_h, fused=fused)


def cpu_run(rs, X, Y, alpha=8, k_h=1, k=None, tau=None):
    return oracle.run_kmerco(rs.reads, rs.offsets, rs.k if k is None else k,
                             rs.tau if tau is None else tau, X, Y, alpha, k_h)


def assert_same(g, c, what=""):
    names = ["words", "distinct", "trust", "err"]
    for n, a, b in zip(names, g[:4], c[:4]):
        a = np.asarray(a, dtype=np.uint64)
        b = np.asarray(b, dtype=np.uint64)
        assert a.shape == b.shape, f"{what} {n}: shape {a.shape} != {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{what} {n}: {len(bad)} mismatches, first at {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    assert g[4] == c[4], f"{what} n_windows {g[4]} != {c[4]}"


def check(rs, X, Y, alpha=8, k_h=1, k=None, tau=None, what="", fused=True):
    print(f"case {what}: {rs.name} X={X} Y={Y} alpha={alpha} k_h={k_h} k={k or rs.k} "
          f"bases={rs.n_bases} path={os.environ.get('KMERCO_PATH', 'auto')} fused={fused}",
          flush=True)
    g = gpu_run(rs, X, Y, alpha, k_h, k, tau, fused)
    c = cpu_run(rs, X, Y, alpha, k_h, k, tau)
    assert_same(g, c, what)
    return g


@pytest.fixture(params=["binned", "direct"])
def path(request, monkeypatch):
    """Insertion path forced for the handles created in the test."""
    monkeypatch.setenv("KMERCO_PATH", request.param)
    return request.param


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def test_tiny_full_size():
    rs = synth.config("tiny")
    X, Y = oracle.dims(rs.n_items)
    g = check(rs, X, Y, what="tiny")
    ref = json.load(open(os.path.join(GOLDEN, "tiny_digests.json")))
    assert (X, Y) == (ref["X"], ref["Y"])
    assert hashlib.sha256(g[0].tobytes()).hexdigest() == ref["words_sha256"]


def test_bacterial_small_scale():
    rs = synth.config("bacterial", scale=0.02)
    X, Y = oracle.dims(rs.n_items)
    check(rs, X, Y, what="bacterial x0.02")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()


def test_bacterial_full_size_digests():
    """The benchmark's workload at full size, in the launch configuration the
    benchmark times, against digests written by tests/golden/make_digests.py
    from the oracle."""
    ref = json.load(open(os.path.join(GOLDEN, "bacterial_digests.json")))
    rs = synth.config("bacterial")
    X, Y = oracle.dims(rs.n_items)
    assert (X, Y) == (ref["X"], ref["Y"]) and rs.n_bases == ref["n_bases"]
    print(f"case bacterial full: X={X} Y={Y} bases={rs.n_bases}", flush=True)
    words, distinct, trust, err, nw = gpu_run(rs, X, Y)
    assert nw == ref["n_windows"]
    assert len(distinct) == ref["n_distinct"]
    assert len(trust) == ref["n_trust"] and len(err) == ref["n_err"]
    assert _sha(words) == ref["words_sha256"]
    assert _sha(distinct) == ref["distinct_sha256"]
    assert _sha(trust) == ref["trust_sha256"]
    assert _sha(err) == ref["err_sha256"]


# ---------------------------------------------------------------------------
# shapes, k, layouts, collisions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 7, 16, 21, 31, 32])
def test_ragged_reads_all_k(k, path):
    rs = synth.random_reads(100 + k, 700, 1, 400, k=k, tau=2, p_n=0.01, p_other=0.005)
    check(rs, 257, 263, k=k, what=f"ragged k={k}")
    check(rs, 257, 263, k=k, what=f"ragged k={k} unfused", fused=False)


@pytest.mark.parametrize("alpha,k_h", [(8, 1), (8, 2), (8, 3), (4, 1), (4, 3), (5, 2), (7, 1),
                                       (12, 2), (16, 1), (21, 1), (32, 2), (1, 1), (3, 8)])
def test_heavy_collisions(alpha, k_h, path):
    """A 3 x 5 filter: every cell is hit thousands of times (contention,
    saturation, first-seen between colliding k-mers)."""
    rs = synth.random_reads(200 + alpha * 10 + k_h, 300, 20, 200, k=9, tau=3, p_n=0.01)
    check(rs, 3, 5, alpha=alpha, k_h=k_h, what=f"collide a={alpha} kh={k_h}")


@pytest.mark.parametrize("alpha,k_h", [(8, 2), (6, 3), (16, 4), (10, 1)])
def test_medium_filters_multi_hash(alpha, k_h, path):
    rs = synth.random_reads(300 + alpha + k_h, 2000, 50, 300, k=25, tau=2, p_n=0.002)
    check(rs, 211, 223, alpha=alpha, k_h=k_h, what=f"medium a={alpha} kh={k_h}")


def test_low_complexity_saturation(path):
    """Two-letter reads: few distinct k-mers, counters saturate."""
    rs = synth.random_reads(401, 3000, 100, 250, k=11, tau=5, alphabet=b"AC")
    check(rs, 101, 103, what="AC alphabet")
    homo = synth.reads_from_strings(["A" * 1000, "T" * 700, "ACGT" * 200], k=21, tau=3)
    check(homo, 7, 11, what="homopolymers")


@pytest.mark.parametrize("k_h", [1, 2])
def test_sparse_and_dense_regions_in_one_call(k_h):
    """A countBF of ~500 regions fed mostly random reads (a few hundred
    entries per region: the sparse per-entry update), plus a homopolymer and
    a periodic read whose k-mers pile thousands of entries onto single
    counters (saturating them) and push their regions past the sparse
    bound (the dense per-counter update)."""
    rnd = synth.random_reads(707 + k_h, 300, 50, 300, k=21, tau=3, p_n=0.01)
    extra = synth.reads_from_strings(["A" * 20000, "ACGT" * 3000, "GATTACA" * 900], k=21, tau=3)
    rs = synth.concat_reads([rnd, extra], name="sparse+dense")
    check(rs, 1009, 1013, k_h=k_h, what=f"sparse+dense kh={k_h}")
    check(rs, 1009, 1013, k_h=k_h, what=f"sparse+dense kh={k_h} unfused", fused=False)


def test_multi_chunk(monkeypatch, path):
    """First-seen resolved in many chunks (chunk size forced small); the
    split of a multi-chunk call is classified after the insert."""
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "2048")
    rs = synth.random_reads(501, 500, 30, 300, k=13, tau=2, alphabet=b"ACGT", p_n=0.01)
    check(rs, 31, 37, k_h=2, what="chunk 2048")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "1024")
    check(rs, 97, 101, what="chunk 1024")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "5000")
    check(rs, 211, 223, what="chunk 4096")


def test_unaligned_reads_pointer():
    rs = synth.random_reads(601, 400, 10, 200, k=17, p_n=0.01)
    reads_pad = torch.zeros(rs.n_bases + 1, dtype=torch.uint8, device="cuda")
    reads_pad[1:] = torch.from_numpy(rs.reads).cuda()
    reads = reads_pad[1:]  # 1-byte offset: the ingest kernel's unaligned path
    offs = torch.from_numpy(rs.offsets.view(np.int64)).cuda()
    g = P.run_kmerco(reads, offs, 17, 2, 59, 61)
    c = cpu_run(rs, 59, 61)
    assert_same(g, c, "unaligned")


# ---------------------------------------------------------------------------
# calls and edge cases
# ---------------------------------------------------------------------------

def test_incremental_equals_concatenated(path):
    parts = [synth.random_reads(700 + i, 200 + 50 * i, 15, 180, k=19, p_n=0.01) for i in range(3)]
    whole = synth.concat_reads(parts)
    X, Y = 61, 67
    bf = P.CountBF(X, Y, 8, 2)
    distinct = torch.empty(whole.n_bases, dtype=torch.int64, device="cuda")
    for p in parts:
        r, o = dev(p)
        bf.insert(r, o, 19, distinct=distinct)
    trust, nt, err, ne = bf.classify(distinct, bf.n_distinct, 2)
    bf.sync()
    nd = int(bf.n_distinct.item())
    u = lambda t: t.cpu().numpy().view(np.uint64)  # noqa: E731
    g = (u(bf.words), u(distinct[:nd]), u(trust[:int(nt.item())]), u(err[:int(ne.item())]),
         int(bf.n_windows.item()))
    c = oracle.run_kmerco(whole.reads, whole.offsets, 19, 2, X, Y, 8, 2)
    assert_same(g, c, "incremental")


def test_resume_from_existing_words(path):
    """kc_create with zero=0 continues an existing countBF (general claim path)."""
    a = synth.random_reads(801, 300, 30, 150, k=15)
    b = synth.random_reads(802, 300, 30, 150, k=15)
    X, Y = 41, 43
    cpu = oracle.CountBF(X, Y, 8, 1)
    cpu.insert(a.reads, a.offsets, 15)
    words = torch.from_numpy(cpu.words.view(np.int64)).cuda()
    bf = P.CountBF(X, Y, 8, 1, words=words, zero=False)
    r, o = dev(b)
    distinct = bf.insert(r, o, 15)
    bf.sync()
    db, _ = cpu.insert(b.reads, b.offsets, 15)
    nd = int(bf.n_distinct.item())
    assert np.array_equal(bf.words.cpu().numpy().view(np.uint64), cpu.words)
    assert np.array_equal(distinct[:nd].cpu().numpy().view(np.uint64), db)


def test_empty_and_degenerate_inputs(path):
    X, Y = 13, 17
    # no bases at all
    bf = P.CountBF(X, Y)
    r = torch.empty(0, dtype=torch.uint8, device="cuda")
    o = torch.zeros(1, dtype=torch.int64, device="cuda")
    bf.insert(r, o, 21)
    bf.sync()
    assert int(bf.n_distinct.item()) == 0 and int(bf.n_windows.item()) == 0
    assert int(bf.words.abs().sum().item()) == 0
    # reads shorter than k, all-N reads, empty reads in between
    rs = synth.reads_from_strings(["ACG", "", "NNNNNNNNNNNNNNNNNNNNNNNN", "ACGTACGTAC", "",
                                   "acgtacgtacgtacgtacgtacgt", "ACGTNACGTACGT"], k=11)
    check(rs, X, Y, what="degenerate")


def test_query_matches_oracle():
    rs = synth.random_reads(901, 500, 30, 200, k=21, p_n=0.01)
    X, Y = 101, 103
    cpu = oracle.CountBF(X, Y, 8, 3)
    d, _ = cpu.insert(rs.reads, rs.offsets, 21)
    rng = np.random.default_rng(3)
    keys = np.concatenate([d, rng.integers(0, 2**42, 500, dtype=np.int64).astype(np.uint64)])
    bf = P.CountBF(X, Y, 8, 3)
    r, o = dev(rs)
    bf.insert(r, o, 21)
    f = bf.query(torch.from_numpy(keys.view(np.int64)).cuda())
    bf.sync()
    assert np.array_equal(f.cpu().numpy().astype(np.uint64), cpu.query(keys))


@pytest.mark.parametrize("tau", [0, 1, 2, 5, 254, 255, 1000])
def test_classify_thresholds(tau):
    rs = synth.random_reads(1001, 800, 30, 200, k=9, alphabet=b"ACGT")
    check(rs, 53, 59, tau=tau, what=f"tau={tau}")
    check(rs, 53, 59, tau=tau, what=f"tau={tau} unfused", fused=False)


def test_large_filter_takes_partitioned_path():
    """A countBF of more than one partition of regions (16448 regions of 2048
    cells at alpha = 8) is binned through partitions automatically."""
    rs = synth.random_reads(1050, 300, 50, 200, k=21, p_n=0.01)
    check(rs, 5801, 5807, what="large filter auto")
    bf = P.CountBF(5801, 5807)
    r, o = dev(rs)
    bf.profile(True)
    bf.insert(r, o, 21)
    phases = bf.profile_read()
    assert "bin_part" in phases and "part_count" in phases, phases


@pytest.mark.parametrize("part_log,alpha,k_h", [(0, 8, 1), (2, 8, 2), (3, 5, 1), (1, 16, 3),
                                                (4, 8, 1)])
def test_partitioned_path_small_partitions(monkeypatch, part_log, alpha, k_h):
    """The partitioned path on small countBFs, with partitions of 2^part_log
    regions (so that many partitions, ragged last ones and empty ones occur)."""
    monkeypatch.setenv("KMERCO_PATH", "binned")
    monkeypatch.setenv("KMERCO_PART_LOG", str(part_log))
    rs = synth.random_reads(1200 + part_log, 2500, 20, 300, k=25, p_n=0.005, tau=2)
    check(rs, 401, 409, alpha=alpha, k_h=k_h, what=f"partitioned part_log={part_log}")
    check(rs, 401, 409, alpha=alpha, k_h=k_h, what=f"partitioned unfused part_log={part_log}",
          fused=False)


@pytest.mark.parametrize("chunk", [1 << 14, 100_000])
def test_partitioned_multi_chunk(monkeypatch, chunk):
    monkeypatch.setenv("KMERCO_PATH", "binned")
    monkeypatch.setenv("KMERCO_PART_LOG", "2")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", str(chunk))
    rs = synth.random_reads(1300, 3000, 20, 250, k=31, p_n=0.002, alphabet=b"ACGT")
    check(rs, 211, 223, what=f"partitioned chunks of {chunk}")
    low = synth.random_reads(1301, 1500, 30, 200, k=13, alphabet=b"AC")  # heavy collisions
    check(low, 211, 223, alpha=4, what=f"partitioned low complexity chunks of {chunk}")


def test_partitioned_bacterial_sample(monkeypatch):
    monkeypatch.setenv("KMERCO_PART_LOG", "3")
    rs = synth.config("bacterial", scale=0.05)
    X, Y = oracle.dims(rs.n_items)
    check(rs, X, Y, what="bacterial x0.05, partitions of 8 regions")


def test_paths_agree_on_bacterial_sample(monkeypatch):
    rs = synth.config("bacterial", scale=0.01)
    X, Y = oracle.dims(rs.n_items)
    monkeypatch.setenv("KMERCO_PATH", "direct")
    a = gpu_run(rs, X, Y)
    monkeypatch.setenv("KMERCO_PATH", "binned")
    b = gpu_run(rs, X, Y)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("X,Y,what", [(4201, 4211, "8638 regions: tiles of 2^17 positions"),
                                      (2621, 2657, "3400 regions: 4096 tiles, 128 slices")])
def test_full_chunk_against_oracle_digests(monkeypatch, X, Y, what):
    """A full binned chunk (2^28 positions) and a tail: the binned entries
    hold positions relative to their tile (level 1) and slice of tiles
    (level 2), so the largest tiles and the most slices a chunk can have are
    checked against the oracle's digests of this seeded input (written by
    tests/golden/make_digests.py), and the direct path against the same."""
    ref = json.load(open(os.path.join(GOLDEN, f"fullchunk_{X}x{Y}_digests.json")))
    rs = synth.random_reads(1500, 1_400_000, 150, 250, k=31, p_n=0.0005, tau=3)
    assert rs.n_bases > (1 << 28) and rs.n_bases == ref["n_bases"]
    assert (X, Y, rs.k, rs.tau) == (ref["X"], ref["Y"], ref["k"], ref["tau"])
    print(f"case full chunk {what}: X={X} Y={Y} bases={rs.n_bases}", flush=True)
    r, o = dev(rs)
    outs = {}
    for p in ("binned", "direct"):
        monkeypatch.setenv("KMERCO_PATH", p)
        print(f"case full chunk {what}: path {p}", flush=True)
        bf = P.CountBF(X, Y)
        bf.profile(True)
        d, t, nt, e, ne = bf.insert_classify(r, o, rs.k, rs.tau)
        bf.sync()
        nd = int(bf.n_distinct.item())
        outs[p] = [bf.words.clone(), d[:nd].clone(), t[:int(nt.item())].clone(),
                   e[:int(ne.item())].clone(), int(bf.n_windows.item())]
        phases = bf.profile_read()
        assert (p == "binned") == ("bin_region" in phases), phases
        assert p == "direct" or phases["bin_region"][1] == 2  # the full chunk and the tail
        bf.close()
        del d, t, e
    for p, (words, distinct, trust, err, nw) in outs.items():
        assert nw == ref["n_windows"], p
        assert (distinct.numel(), trust.numel(), err.numel()) == \
            (ref["n_distinct"], ref["n_trust"], ref["n_err"]), p
        assert _sha(words.cpu().numpy()) == ref["words_sha256"], p
        assert _sha(distinct.cpu().numpy()) == ref["distinct_sha256"], p
        assert _sha(trust.cpu().numpy()) == ref["trust_sha256"], p
        assert _sha(err.cpu().numpy()) == ref["err_sha256"], p
    a, b = outs["binned"], outs["direct"]
    for n, x, y in zip(["words", "distinct", "trust", "err"], a[:4], b[:4]):
        assert torch.equal(x, y), f"{what} {n} differs"


def test_small_chunk_spread_over_many_workgroups():
    """About 9 M positions: the binned path hashes them in tiles of 4608
    positions (between the 4096 floor and the 65536 of large chunks), about
    1950 workgroups; all outputs against the oracle."""
    rs = synth.random_reads(1600, 60_000, 100, 200, k=27, p_n=0.002, tau=2)
    assert 8_000_000 < rs.n_bases < 10_000_000
    X, Y = oracle.dims(rs.n_items)
    check(rs, X, Y, what="9 M positions, small tiles")


def test_errors_and_capacity():
    rs = synth.random_reads(1101, 100, 30, 100, k=21)
    r, o = dev(rs)
    bf = P.CountBF(29, 31)
    small = torch.empty(5, dtype=torch.int64, device="cuda")
    bf.insert(r, o, 21, distinct=small)
    with pytest.raises(P.KmercoError) as e:
        bf.sync()
    assert e.value.status == -3
    c = cpu_run(rs, 29, 31)
    assert int(bf.n_distinct.item()) == len(c[1])  # the count reports the need
    assert np.array_equal(small.cpu().numpy().view(np.uint64), c[1][:5])
    with pytest.raises(P.KmercoError) as e:
        bf.insert(r, o, 23)  # k differs from the first insert
    assert e.value.status == -5
    bf.sync()  # sticky status was cleared


def test_repeatable():
    rs = synth.random_reads(1201, 1000, 50, 250, k=31, p_n=0.01)
    a = gpu_run(rs, 89, 97, k_h=2)
    b = gpu_run(rs, 89, 97, k_h=2)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


def test_large_full_size_digests():
    """The large workload at full size: 8 Gbases of reads into an 8 GB
    countBF (the partitioned binned path, several chunks), against the
    oracle's digests."""
    path = os.path.join(GOLDEN, "large_digests.json")
    if not os.path.exists(path):
        pytest.skip("no oracle digests for the large workload")
    ref = json.load(open(path))
    print("case large full size: generating reads", flush=True)
    rs = synth.config("large")
    assert rs.n_bases == ref["n_bases"]
    X, Y = ref["X"], ref["Y"]
    r, o = dev(rs)
    del rs
    room = ref["n_distinct"] + 1024
    out = {n: torch.empty(room, dtype=torch.int64, device="cuda") for n in ("d", "t", "e")}
    bf = P.CountBF(X, Y)
    print(f"case large full size: insert+classify X={X} Y={Y}", flush=True)
    _, _, n_trust, _, n_err = bf.insert_classify(r, o, ref["k"], ref["tau"], distinct=out["d"],
                                                 trust=out["t"], err=out["e"])
    bf.sync()
    del r, o
    nd, nt, ne = int(bf.n_distinct.item()), int(n_trust.item()), int(n_err.item())
    assert int(bf.n_windows.item()) == ref["n_windows"]
    assert (nd, nt, ne) == (ref["n_distinct"], ref["n_trust"], ref["n_err"])

    def h(t):
        return hashlib.sha256(t.cpu().numpy().view(np.uint64).tobytes()).hexdigest()

    assert h(bf.words) == ref["words_sha256"]
    assert h(out["d"][:nd]) == ref["distinct_sha256"]
    assert h(out["t"][:nt]) == ref["trust_sha256"]
    assert h(out["e"][:ne]) == ref["err_sha256"]
    bf.close()


def test_bacterial_k55_full_size_digests():
    """The bacterial workload's reads at k = 55 (two-word keys, the paper's
    longer k-mers) at full size, in the benchmark's launch configuration,
    against the oracle's digests."""
    ref = json.load(open(os.path.join(GOLDEN, "bacterial_k55_digests.json")))
    rs = synth.config("bacterial")
    X, Y = oracle.dims(rs.n_items)
    assert (X, Y, 55) == (ref["X"], ref["Y"], ref["k"]) and rs.n_bases == ref["n_bases"]
    print(f"case bacterial k=55 full: X={X} Y={Y} bases={rs.n_bases}", flush=True)
    words, distinct, trust, err, nw = gpu_run(rs, X, Y, k=55)
    assert nw == ref["n_windows"]
    assert (len(distinct), len(trust), len(err)) == \
        (ref["n_distinct"], ref["n_trust"], ref["n_err"])
    assert _sha(words) == ref["words_sha256"]
    assert _sha(distinct) == ref["distinct_sha256"]
    assert _sha(trust) == ref["trust_sha256"]
    assert _sha(err) == ref["err_sha256"]


# ---------------------------------------------------------------------------
# regions of 8192 counters (the region pass's smaller LDS tile)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,k_h", [(8, 1), (8, 2), (5, 1), (16, 3), (4, 1), (32, 1)])
def test_small_regions(monkeypatch, alpha, k_h):
    """Regions of 8192 counters on both binned paths: sparse and dense
    regions, heavy collisions, several chunks, fused and unfused split."""
    monkeypatch.setenv("KMERCO_REGION_COUNTERS", "8192")
    rnd = synth.random_reads(2700 + alpha + k_h, 400, 50, 300, k=21, tau=3, p_n=0.01)
    extra = synth.reads_from_strings(["A" * 9000, "ACGT" * 2000], k=21, tau=3)
    rs = synth.concat_reads([rnd, extra], name="small regions")
    check(rs, 1009, 1013, alpha=alpha, k_h=k_h, what=f"small regions a={alpha} kh={k_h}")
    check(rs, 1009, 1013, alpha=alpha, k_h=k_h, what="small regions unfused", fused=False)
    check(rs, 3, 5, alpha=alpha, k_h=k_h, what="small regions, 3x5 filter")
    monkeypatch.setenv("KMERCO_PART_LOG", "2")
    check(rs, 401, 409, alpha=alpha, k_h=k_h, what="small regions, partitions of 4")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "50000")
    check(rs, 401, 409, alpha=alpha, k_h=k_h, what="small regions, partitioned chunks")


def test_small_regions_bacterial_sample(monkeypatch):
    monkeypatch.setenv("KMERCO_REGION_COUNTERS", "8192")
    rs = synth.config("bacterial", scale=0.05)
    X, Y = oracle.dims(rs.n_items)
    check(rs, X, Y, what="bacterial x0.05, regions of 8192 counters")
    monkeypatch.setenv("KMERCO_PART_LOG", "3")
    check(rs, X, Y, what="bacterial x0.05, regions of 8192 counters, partitions of 8")


# ---------------------------------------------------------------------------
# first-seen records turned into flag bytes by the winner passes (the mode of
# chunks beyond 2^28 positions, forced here on small inputs)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,k_h,counters", [(8, 1, "16384"), (8, 2, "16384"), (5, 1, "8192"),
                                                (16, 3, "16384"), (4, 1, "8192")])
def test_winner_records(monkeypatch, alpha, k_h, counters):
    monkeypatch.setenv("KMERCO_WINNER_RECORDS", "1")
    monkeypatch.setenv("KMERCO_REGION_COUNTERS", counters)
    rnd = synth.random_reads(2900 + alpha + k_h, 600, 50, 300, k=23, tau=2, p_n=0.01)
    extra = synth.reads_from_strings(["A" * 9000, "ACGT" * 2000, "GATTACA" * 500], k=23, tau=2)
    rs = synth.concat_reads([rnd, extra], name="winner records")
    check(rs, 1009, 1013, alpha=alpha, k_h=k_h, what=f"records a={alpha} kh={k_h}")
    check(rs, 1009, 1013, alpha=alpha, k_h=k_h, what="records unfused", fused=False)
    check(rs, 3, 5, alpha=alpha, k_h=k_h, what="records, 3x5 filter")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "40000")
    check(rs, 1009, 1013, alpha=alpha, k_h=k_h, what="records, chunks of 40000")
    monkeypatch.setenv("KMERCO_PART_LOG", "2")
    check(rs, 401, 409, alpha=alpha, k_h=k_h, what="records, partitioned chunks")


def test_winner_records_bacterial_and_wide(monkeypatch):
    monkeypatch.setenv("KMERCO_WINNER_RECORDS", "1")
    rs = synth.config("bacterial", scale=0.05)
    X, Y = oracle.dims(rs.n_items)
    check(rs, X, Y, what="records, bacterial x0.05")
    check(rs, X, Y, k=45, what="records, bacterial x0.05, k=45")
    monkeypatch.setenv("KMERCO_PART_LOG", "3")
    check(rs, X, Y, what="records, bacterial x0.05, partitions of 8")


# ---------------------------------------------------------------------------
# carried classification: a multi-chunk split insert with one hash function
# classifies the earlier chunks' first-seen k-mers in the last chunk's region
# pass (KMERCO_CARRY=0: by the pass that rereads their counters instead)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,counters,part_log",
                         [(8, "16384", "14"), (8, "16384", "2"), (5, "8192", "14"),
                          (4, "8192", "2"), (16, "16384", "14")])
def test_carried_classification(monkeypatch, alpha, counters, part_log):
    monkeypatch.setenv("KMERCO_REGION_COUNTERS", counters)
    monkeypatch.setenv("KMERCO_PART_LOG", part_log)
    rnd = synth.random_reads(3100 + alpha, 700, 50, 300, k=23, tau=2, p_n=0.01)
    extra = synth.reads_from_strings(["A" * 9000, "ACGT" * 2000, "GATTACA" * 500], k=23, tau=2)
    rs = synth.concat_reads([rnd, extra], name="carried")
    X, Y = (401, 409) if part_log == "2" else (1009, 1013)
    for chunk in ("40000", "16384", "1024"):
        monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", chunk)
        bf = P.CountBF(X, Y, alpha, 1)
        plan = bf.plan(rs.n_bases)
        bf.close()
        assert plan["n_chunks"] > 2
        # eta >= 8 carries (the region's cells fit the staged-cell array)
        assert plan["carried"] == (1 if 64 // alpha >= 8 else 0), plan
        outs = []
        for carry in ("1", "0"):
            monkeypatch.setenv("KMERCO_CARRY", carry)
            outs.append(check(rs, X, Y, alpha=alpha, what=f"carry={carry} chunks of {chunk}"))
        for a, b in zip(outs[0][:4], outs[1][:4]):
            assert np.array_equal(a, b)
        monkeypatch.setenv("KMERCO_WINNER_RECORDS", "1")  # the last chunk's own records too
        check(rs, X, Y, alpha=alpha, what=f"carried, records mode, chunks of {chunk}")
        check(rs, X, Y, alpha=alpha, k=45, what=f"carried, k=45, chunks of {chunk}")
        monkeypatch.delenv("KMERCO_WINNER_RECORDS")
        monkeypatch.delenv("KMERCO_CARRY")


@pytest.mark.parametrize("X,Y,chunk", [(211, 223, 40000), (101, 103, 65536)])
def test_carried_classification_many_records_per_region(monkeypatch, X, Y, chunk):
    """More than 1024 first-seen records of an earlier chunk in one region
    (sparse regions at 211 x 223, dense ones at 101 x 103): the last chunk's
    region pass marks the first 1024 from the records it requested with the
    region and the others in a loop."""
    n_first = chunk // 300 - 1  # reads wholly inside the first chunk
    first = synth.random_reads(3300 + X, n_first, 300, 300, k=23, tau=2)
    rest = synth.random_reads(3400 + X, 3 * n_first, 300, 300, k=23, tau=2)
    rs = synth.concat_reads([first, rest], name="carried, many records")
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", str(chunk))
    bf = P.CountBF(X, Y, 8, 1)
    plan = bf.plan(rs.n_bases)
    bf.close()
    assert plan["carried"] == 1 and plan["n_chunks"] >= 3, plan
    # the first chunk's first-seen k-mers (those of the reads inside it, a
    # lower bound) average more than 1024 per region
    n_first_seen = len(cpu_run(first, X, Y)[1])
    assert n_first_seen > 1024 * plan["n_regions"], (n_first_seen, plan)
    check(rs, X, Y, what=f"carried, many records per region, {X}x{Y}, chunks of {chunk}")
    monkeypatch.setenv("KMERCO_WINNER_RECORDS", "1")
    check(rs, X, Y, what=f"carried, many records per region, records mode, {X}x{Y}")


def test_carried_classification_bacterial_sample(monkeypatch):
    rs = synth.config("bacterial", scale=0.05)
    X, Y = oracle.dims(rs.n_items)
    monkeypatch.setenv("KMERCO_CHUNK_POSITIONS", "1000000")
    check(rs, X, Y, what="carried, bacterial x0.05, chunks of 1M")
    monkeypatch.setenv("KMERCO_PART_LOG", "3")
    check(rs, X, Y, what="carried, bacterial x0.05, partitions of 8, chunks of 1M")
