"""Seeded synthetic read sets standing in for the paper's sequencing data.

The paper measures on trimmed SRA read files of four mammals (Experiments,
dataset table).  Those files are not available, so every workload here is
simulated: a random genome, reads sampled at uniform positions from a random
strand, then sequencing errors (substitutions, indels, 'N' calls).

Reads are returned as one concatenated ``uint8`` ASCII buffer plus ``uint64``
CSR offsets (``offsets[0] == 0``, read ``r`` is ``reads[offsets[r]:offsets[r+1]]``).

Nothing here extracts, encodes or hashes k-mers; reverse-complementing a
sampled fragment only simulates reading the opposite strand.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# code -> ASCII byte; code 4 is an 'N' call
_ASCII = np.frombuffer(b"ACGTN", dtype=np.uint8)

# sizing convention: the countBF is sized for about twice the expected number
# of distinct canonical k-mers
SIZING_FACTOR = 2.0


@dataclass
class ReadSet:
    name: str
    reads: np.ndarray          # uint8 ASCII, all reads concatenated
    offsets: np.ndarray        # uint64, n_reads + 1 CSR offsets
    k: int
    tau: int
    n_items: float             # item count the countBF is sized for
    meta: dict = field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_bases(self) -> int:
        return int(self.offsets[-1])

    def subset(self, first: int, count: int, name: str | None = None) -> "ReadSet":
        """Reads ``first .. first+count-1`` as a new set (offsets rebased)."""
        lo = int(self.offsets[first])
        hi = int(self.offsets[first + count])
        offs = (self.offsets[first:first + count + 1] - np.uint64(lo)).astype(np.uint64)
        return ReadSet(name or f"{self.name}[{first}:{first + count}]",
                       self.reads[lo:hi].copy(), offs, self.k, self.tau,
                       self.n_items, dict(self.meta))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def _genome(rng: np.random.Generator, size: int) -> np.ndarray:
    """Uniform i.i.d. ACGT genome (GC 50%) as codes 0..3."""
    return rng.integers(0, 4, size=size, dtype=np.uint8)


def _add_duplications(rng, genome, fraction, min_len, max_len):
    """Overwrite ``fraction`` of the genome with copies of other segments."""
    g = len(genome)
    target = int(fraction * g)
    done = 0
    while done < target:
        ln = int(rng.integers(min_len, max_len + 1))
        src = int(rng.integers(0, g - ln + 1))
        dst = int(rng.integers(0, g - ln + 1))
        genome[dst:dst + ln] = genome[src:src + ln].copy()
        done += ln
    return genome


def _add_repeat_families(rng, genome, fraction, copy_lo, copy_hi, div_lo, div_hi,
                         unit_lo=1000, unit_hi=10000):
    """Cover ``fraction`` of the genome with diverged repeat copies.

    Each family is a random unit placed ``copy_lo..copy_hi`` times; every copy
    carries its own i.i.d. substitutions at a per-family divergence drawn
    uniformly from ``[div_lo, div_hi]``.
    """
    g = len(genome)
    target = int(fraction * g)
    done = 0
    while done < target:
        ln = int(rng.integers(unit_lo, unit_hi + 1))
        unit = rng.integers(0, 4, size=ln, dtype=np.uint8)
        copies = int(rng.integers(copy_lo, copy_hi + 1))
        div = float(rng.uniform(div_lo, div_hi))
        for _ in range(copies):
            c = unit.copy()
            m = rng.random(ln) < div
            c[m] = (c[m] + rng.integers(1, 4, size=int(m.sum()), dtype=np.uint8)) % 4
            dst = int(rng.integers(0, g - ln + 1))
            genome[dst:dst + ln] = c
            done += ln
            if done >= target:
                break
    return genome


def _bernoulli_positions(rng, total: int, p: float) -> np.ndarray:
    """Positions of a Bernoulli(p) process on [0, total) (geometric gaps)."""
    if p <= 0.0 or total <= 0:
        return np.zeros(0, dtype=np.int64)
    out = []
    pos = -1
    mean = total * p
    batch = int(mean + 10.0 * math.sqrt(mean) + 64)
    while True:
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        cand = pos + np.cumsum(gaps)
        keep = cand[cand < total]
        out.append(keep)
        if len(keep) < len(cand):
            break
        pos = int(cand[-1])
    return np.concatenate(out)


def _gather_reads(genome, starts, rev, lengths, offsets, codes):
    """codes[offsets[r]:offsets[r+1]] = genome[starts[r]:starts[r]+lengths[r]],
    or its reverse complement where rev[r]."""
    g = len(genome)
    n = len(lengths)
    if n == 0:
        return
    lmax = int(lengths.max())
    # forward genome, then its reverse complement, then room for the last row;
    # the reverse strand of genome[s:s+L] is (reverse complement)[g-s-L : g-s]
    both = np.concatenate([genome, (3 - genome[::-1]).astype(np.uint8),
                           np.zeros(lmax, dtype=np.uint8)])
    rows = np.lib.stride_tricks.sliding_window_view(both, lmax)
    src = np.where(rev, g + (g - starts - lengths), starts)
    col = np.arange(lmax, dtype=np.int64)[None, :]
    step = 262_144
    for a in range(0, n, step):
        b = min(n, a + step)
        block = rows[src[a:b]]
        codes[int(offsets[a]):int(offsets[b])] = block[col < lengths[a:b, None]]


def _sample_reads(rng, genome, lengths, p_sub=0.0, p_indel=0.0, p_n=0.0):
    """Sample reads of the given lengths; returns (codes uint8, offsets uint64).

    Each read starts at a uniform position, comes from the reverse strand with
    probability 1/2, then gets indels (per-base rate ``p_indel``, read length
    kept), substitutions to one of the three other bases (rate ``p_sub``) and
    'N' calls (rate ``p_n``).
    """
    g = len(genome)
    lengths = np.asarray(lengths, dtype=np.int64)
    n = len(lengths)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    codes = np.empty(total, dtype=np.uint8)
    margin = 64  # room for deletions
    starts = rng.integers(0, g - lengths - margin + 1)
    rev = rng.random(n) < 0.5
    _gather_reads(genome, starts, rev, lengths, offsets, codes)
    if p_indel > 0.0:
        events = rng.binomial(lengths, p_indel)
        for r in np.nonzero(events)[0]:
            ln = int(lengths[r])
            s = int(starts[r])
            frag = genome[s:s + ln + margin].copy()
            if rev[r]:
                frag = (3 - frag[::-1]).astype(np.uint8)
            seq = list(frag)
            for _ in range(int(events[r])):
                pos = int(rng.integers(0, ln))
                if rng.random() < 0.5:
                    del seq[pos]
                else:
                    seq.insert(pos, int(rng.integers(0, 4)))
            o = int(offsets[r])
            codes[o:o + ln] = np.asarray(seq[:ln], dtype=np.uint8)
    if p_sub > 0.0:
        pos = _bernoulli_positions(rng, total, p_sub)
        codes[pos] = (codes[pos] + rng.integers(1, 4, size=len(pos), dtype=np.uint8)) % 4
    if p_n > 0.0:
        pos = _bernoulli_positions(rng, total, p_n)
        codes[pos] = 4
    return codes, offsets


def _to_ascii(codes: np.ndarray) -> np.ndarray:
    return _ASCII[codes]


def _expected_distinct(genome_len: int, n_bases: int, p_err: float, k: int) -> float:
    """Rough expected distinct canonical k-mers: the genome's own k-mers plus
    up to ``k`` novel k-mers per sequencing error."""
    return float(genome_len + n_bases * p_err * k)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def _cfg_tiny(scale: float) -> ReadSet:
    """100 kbp uniform genome, 10,000 x 100 bp reads, 1% substitutions, k=21."""
    rng = np.random.default_rng(1001)
    g = max(1000, int(100_000 * scale))
    n = max(1, int(10_000 * scale))
    genome = _genome(rng, g)
    codes, offs = _sample_reads(rng, genome, np.full(n, 100), p_sub=0.01)
    d = _expected_distinct(g, n * 100, 0.01, 21)
    return ReadSet("tiny", _to_ascii(codes), offs, 21, 2, SIZING_FACTOR * d,
                   {"genome": g, "reads": n, "read_len": 100, "p_sub": 0.01})


def _cfg_bacterial(scale: float) -> ReadSet:
    """5 Mbp genome (2% duplicated 1-5 kbp segments), 1.0 M x 150 bp reads at
    30x, 0.5% substitutions + 0.05% indels + 0.1% N, k=31."""
    rng = np.random.default_rng(1002)
    g = max(20_000, int(5_000_000 * scale))
    n = max(1, int(1_000_000 * scale))
    genome = _add_duplications(rng, _genome(rng, g), 0.02, 1000, 5000)
    codes, offs = _sample_reads(rng, genome, np.full(n, 150),
                                p_sub=0.005, p_indel=0.0005, p_n=0.001)
    d = _expected_distinct(g, n * 150, 0.0055, 31)
    return ReadSet("bacterial", _to_ascii(codes), offs, 31, 3, SIZING_FACTOR * d,
                   {"genome": g, "reads": n, "read_len": 150, "p_sub": 0.005,
                    "p_indel": 0.0005, "p_n": 0.001})


def _cfg_batched(scale: float, n_sets: int = 256, first: int | None = None) -> list[ReadSet]:
    """256 independent sets: read counts lognormal (median 20k, clipped to
    1k..500k), read lengths U[50, 300], k in {21, 25, 31}, substitution rate
    U[0.1%, 2%], each from its own uniform genome at about 20x coverage.
    ``first`` builds only the first sets (the same ones: each set draws from
    its own seed)."""
    seeds = np.random.SeedSequence(1003).spawn(n_sets)
    out = []
    for s, ss in enumerate(seeds[:first]):
        rng = np.random.default_rng(ss)
        n = int(np.clip(round(rng.lognormal(math.log(20_000), 1.0)), 1_000, 500_000))
        n = max(1, int(n * scale))
        k = int(rng.choice([21, 25, 31]))
        err = float(rng.uniform(0.001, 0.02))
        lengths = rng.integers(50, 301, size=n)
        g = max(2_000, int(lengths.sum() / 20))
        genome = _genome(rng, g)
        codes, offs = _sample_reads(rng, genome, lengths, p_sub=err)
        d = _expected_distinct(g, int(lengths.sum()), err, k)
        out.append(ReadSet(f"batched/{s}", _to_ascii(codes), offs, k, 2,
                           SIZING_FACTOR * d,
                           {"genome": g, "reads": n, "p_sub": err}))
    return out


def _cfg_large(scale: float) -> ReadSet:
    """200 Mbp genome with 30% diverged repeats (copy number 2-50, 1-10%
    divergence), 32 M x 250 bp reads (40x), 0.3% substitutions, k=31; the
    countBF is about 8 GB (n_items chosen so that sqrt(m/128) ~ 31623)."""
    rng = np.random.default_rng(1004)
    g = max(50_000, int(200_000_000 * scale))
    n = max(1, int(32_000_000 * scale))
    genome = _add_repeat_families(rng, _genome(rng, g), 0.30, 2, 50, 0.01, 0.10)
    codes, offs = _sample_reads(rng, genome, np.full(n, 250), p_sub=0.003)
    n_items = 8.9e9 * scale
    return ReadSet("large", _to_ascii(codes), offs, 31, 5, n_items,
                   {"genome": g, "reads": n, "read_len": 250, "p_sub": 0.003})


_WORKLOADS = {
    "tiny": _cfg_tiny,
    "bacterial": _cfg_bacterial,
    "batched": _cfg_batched,
    "large": _cfg_large,
}


def config_names():
    return list(_WORKLOADS)


def config(name: str, scale: float = 1.0):
    """Build a workload by name (``tiny``, ``bacterial``, ``batched``, ``large``).

    ``scale`` shrinks genome and read counts proportionally (tests use small
    scales); the seeds do not depend on it.
    """
    return _WORKLOADS[name](scale)


# ---------------------------------------------------------------------------
# ad-hoc inputs for edge-case tests
# ---------------------------------------------------------------------------

def reads_from_strings(seqs, k=21, tau=2, n_items=1000.0, name="strings") -> ReadSet:
    bufs = [s.encode("ascii") if isinstance(s, str) else bytes(s) for s in seqs]
    offs = np.zeros(len(bufs) + 1, dtype=np.uint64)
    np.cumsum([len(b) for b in bufs], out=offs[1:])
    reads = np.frombuffer(b"".join(bufs), dtype=np.uint8).copy()
    return ReadSet(name, reads, offs, k, tau, n_items)


def random_reads(seed: int, n_reads: int, min_len: int, max_len: int, k: int = 21,
                 tau: int = 2, p_n: float = 0.0, p_other: float = 0.0,
                 alphabet: bytes = b"ACGT", n_items: float | None = None) -> ReadSet:
    """Independent random reads (no genome) with ragged lengths.

    ``p_n`` puts 'N' calls, ``p_other`` puts bytes outside ACGT (lower case,
    IUPAC codes, punctuation) to exercise invalid-base handling.  A small
    ``alphabet`` (e.g. ``b"AC"``) makes repeated k-mers and collisions common.
    """
    rng = np.random.default_rng(seed)
    lengths = rng.integers(min_len, max_len + 1, size=n_reads)
    offs = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offs[1:])
    total = int(offs[-1])
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    reads = alpha[rng.integers(0, len(alpha), size=total)]
    if p_n > 0:
        reads[rng.random(total) < p_n] = ord("N")
    if p_other > 0:
        others = np.frombuffer(b"acgtnRYKM-.*", dtype=np.uint8)
        m = rng.random(total) < p_other
        reads[m] = others[rng.integers(0, len(others), size=int(m.sum()))]
    if n_items is None:
        n_items = 2.0 * max(1, total)
    return ReadSet(f"random/{seed}", reads, offs, k, tau, float(n_items))


def concat_reads(sets, name="concat") -> ReadSet:
    """Concatenate read sets (the first set's k, tau and n_items are kept)."""
    reads = np.concatenate([s.reads for s in sets])
    offs = [np.zeros(1, dtype=np.uint64)]
    base = 0
    for s in sets:
        offs.append(s.offsets[1:] + np.uint64(base))
        base += s.n_bases
    return ReadSet(name, reads, np.concatenate(offs).astype(np.uint64),
                   sets[0].k, sets[0].tau, sets[0].n_items)
