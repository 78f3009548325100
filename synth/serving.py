"""Seeded request trace for the serving form.

Sixteen genomes (sizes log-uniform in 1-20 Mbp, uniform ACGT), one session
per genome with its own k drawn from {21, 31}.  Requests arrive as a Poisson
process (mean rate 50/s); each picks a genome uniformly, carries a read set
of n reads (n log-uniform in 10k-2M, scaled), read lengths uniform in
100-250, 0.5% substitutions, and is an insert, or with probability 1/4 an
insert followed by a classification of the session's distinct k-mers at a
threshold drawn from 2..5.

Reads come from one pool per genome, as many reads as the genome's largest
request; a request takes a contiguous run of pool reads at a uniform start,
so requests of one session can share reads (the counts then grow as for
repeated sequencing of the same library).  Pools are sampled with
``sample_reads_fast``: the same read model as the other workloads without
indels and 'N' calls, vectorised for the multi-gigabase pools.

Nothing here extracts, encodes or hashes k-mers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .reads import (_ASCII, SIZING_FACTOR, _bernoulli_positions, _expected_distinct,
                    _gather_reads, _genome)


def sample_reads_fast(rng, genome: np.ndarray, lengths: np.ndarray, p_sub: float):
    """Reads of the given lengths at uniform starts, reverse strand with
    probability 1/2, i.i.d. substitutions to one of the other three bases;
    returns (ASCII uint8, offsets uint64)."""
    g = len(genome)
    lengths = np.asarray(lengths, dtype=np.int64)
    n = len(lengths)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    starts = rng.integers(0, g - lengths + 1)
    rev = rng.random(n) < 0.5
    codes = np.empty(total, dtype=np.uint8)
    _gather_reads(genome, starts, rev, lengths, offsets, codes)
    pos = _bernoulli_positions(rng, total, p_sub)
    codes[pos] = (codes[pos] + rng.integers(1, 4, size=len(pos), dtype=np.uint8)) % 4
    return _ASCII[codes], offsets


@dataclass
class Request:
    t: float          # arrival time (s)
    genome: int       # session index
    first_read: int   # run of pool reads
    n_reads: int
    classify: bool
    tau: int


@dataclass
class ServingWorkload:
    genome_sizes: list
    ks: list                     # per session
    pools: list                  # per genome: (reads uint8, offsets uint64)
    requests: list               # Request, in arrival order
    n_items: list                # per session: countBF sizing (2x expected distinct)
    expected_distinct: list      # per session
    meta: dict = field(default_factory=dict)

    def request_reads(self, i: int):
        """(reads, offsets with offsets[0] == 0) of request i (views/copies)."""
        q = self.requests[i]
        reads, offs = self.pools[q.genome]
        lo = int(offs[q.first_read])
        hi = int(offs[q.first_read + q.n_reads])
        return reads[lo:hi], (offs[q.first_read:q.first_read + q.n_reads + 1]
                              - np.uint64(lo)).astype(np.uint64)

    def request_bases(self, i: int) -> int:
        q = self.requests[i]
        offs = self.pools[q.genome][1]
        return int(offs[q.first_read + q.n_reads]) - int(offs[q.first_read])


def serving_workload(scale: float = 1.0, duration_s: float = 5.0, rate: float = 50.0,
                     n_genomes: int = 16, p_sub: float = 0.005,
                     seed: int = 1005) -> ServingWorkload:
    """The trace and read pools.  ``scale`` shrinks genome sizes and read
    counts together; the arrival process does not depend on it."""
    rng = np.random.default_rng(seed)
    sizes = [max(5_000, int(round(math.exp(rng.uniform(math.log(1e6), math.log(2e7))) * scale)))
             for _ in range(n_genomes)]
    ks = [int(rng.choice([21, 31])) for _ in range(n_genomes)]
    # arrivals
    reqs = []
    t = 0.0
    lo, hi = math.log(10_000), math.log(2_000_000)
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        g = int(rng.integers(0, n_genomes))
        n = max(1, int(round(math.exp(rng.uniform(lo, hi)) * scale)))
        cls = bool(rng.random() < 0.25)
        tau = int(rng.integers(2, 6))
        reqs.append(Request(t, g, 0, n, cls, tau))
    # pools sized to each genome's largest request; request starts in them
    pools = []
    for g in range(n_genomes):
        grng = np.random.default_rng(np.random.SeedSequence([seed, g]))
        genome = _genome(grng, sizes[g])
        mine = [q for q in reqs if q.genome == g]
        n_pool = max([q.n_reads for q in mine], default=1)
        lengths = grng.integers(100, 251, size=n_pool)
        reads, offs = sample_reads_fast(grng, genome, lengths, p_sub)
        pools.append((reads, offs))
        for q in mine:
            q.first_read = int(grng.integers(0, n_pool - q.n_reads + 1))
    # per-session sizing from the session's planned volume (closed form)
    ws = ServingWorkload(sizes, ks, pools, reqs, [], [],
                         {"duration_s": duration_s, "rate": rate, "p_sub": p_sub,
                          "scale": scale})
    vol = [0] * n_genomes
    for i, q in enumerate(reqs):
        vol[q.genome] += ws.request_bases(i)
    for g in range(n_genomes):
        d = _expected_distinct(sizes[g], vol[g], p_sub, ks[g])
        ws.expected_distinct.append(d)
        ws.n_items.append(SIZING_FACTOR * d)
    return ws
