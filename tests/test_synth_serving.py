"""The serving trace generator: read model, sizes and determinism (host only)."""
import math

import numpy as np

import synth

_RC = bytes.maketrans(b"ACGT", b"TGCA")


def test_fast_sampler_reads_are_genome_substrings():
    rng = np.random.default_rng(5)
    genome = rng.integers(0, 4, size=3000).astype(np.uint8)
    lengths = rng.integers(100, 251, size=400)
    reads, offs = synth.sample_reads_fast(rng, genome, lengths, p_sub=0.0)
    g = np.frombuffer(b"ACGT", dtype=np.uint8)[genome].tobytes()
    rc = g.translate(_RC)[::-1]
    assert np.array_equal(np.diff(offs.astype(np.int64)), lengths)
    fwd = 0
    for r in range(len(lengths)):
        s = reads[int(offs[r]):int(offs[r + 1])].tobytes()
        assert s in g or s in rc, f"read {r}"
        fwd += s in g
    assert 150 < fwd < 250  # strand is a fair coin


def test_fast_sampler_substitution_rate():
    rng = np.random.default_rng(6)
    genome = rng.integers(0, 4, size=20000).astype(np.uint8)
    lengths = np.full(2000, 200)
    reads, offs = synth.sample_reads_fast(rng, genome, lengths, p_sub=0.01)
    g = np.frombuffer(b"ACGT", dtype=np.uint8)[genome].tobytes()
    rc = g.translate(_RC)[::-1]
    clean = sum(reads[int(offs[r]):int(offs[r + 1])].tobytes() in g
                or reads[int(offs[r]):int(offs[r + 1])].tobytes() in rc for r in range(2000))
    expect = 2000 * (1 - 0.01) ** 200  # reads without a substitution
    assert abs(clean - expect) < 5 * math.sqrt(expect)
    assert set(np.unique(reads)) <= set(b"ACGT")


def test_trace_shape_and_determinism():
    a = synth.serving_workload(scale=0.002, duration_s=4.0)
    b = synth.serving_workload(scale=0.002, duration_s=4.0)
    n = len(a.requests)
    assert abs(n - 200) < 5 * math.sqrt(200)  # Poisson(50/s) over 4 s
    t = [q.t for q in a.requests]
    assert t == sorted(t) and t[-1] < 4.0
    assert [(q.t, q.genome, q.first_read, q.n_reads, q.classify, q.tau) for q in a.requests] == \
        [(q.t, q.genome, q.first_read, q.n_reads, q.classify, q.tau) for q in b.requests]
    assert all(np.array_equal(x[0], y[0]) for x, y in zip(a.pools, b.pools))
    assert set(a.ks) <= {21, 31} and len(a.genome_sizes) == 16
    for i, q in enumerate(a.requests):
        assert 2 <= q.tau <= 5
        assert max(1, round(10_000 * 0.002)) <= q.n_reads <= round(2_000_000 * 0.002)
        reads, offs = a.request_reads(i)
        assert offs[0] == 0 and len(offs) == q.n_reads + 1 and int(offs[-1]) == len(reads)
        lens = np.diff(offs.astype(np.int64))
        assert lens.min() >= 100 and lens.max() <= 250
    frac = np.mean([q.classify for q in a.requests])
    assert 0.1 < frac < 0.4
    for g in range(16):
        assert a.n_items[g] == 2 * a.expected_distinct[g] >= 2 * a.genome_sizes[g]
