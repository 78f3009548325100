"""Accuracy and placement of KmerCo on synthetic data: the paper's data set
analysis (Sec. 4.3) and countBF-size experiments (the supplement's "varying
countBF data structure size" table) on the synthetic stand-ins.

For each countBF size the GPU path inserts and classifies the workload, and
its distinct, trustworthy and erroneous lists are compared with exact k-mer
counts; the insertion rate is timed with the reads resident in HBM.  Exact
counts are plain numpy: the 2-bit key of every valid window (inside one
read, only A/C/G/T), the strand-independent form min(key, reverse
complement), np.unique.  KmerCo's lists hold the strand its hash picks
(Sec. 2.3), so they are compared in that same strand-independent form.

Usage: python -m paper_2305_07545_amd.evaluate [--workload bacterial]
       [--scale 0.1] [--sizes 0.125,0.5,1,4,16] [--steps 5]   (one JSON line per size)
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

# A C G T -> 0 1 2 3; every other byte invalid (255)
_CODE = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i


def window_keys(reads: np.ndarray, offsets: np.ndarray, k: int) -> np.ndarray:
    """Forward 2-bit keys (first base most significant) of the valid windows,
    in read order and increasing start position."""
    n = len(reads)
    if n < k:
        return np.zeros(0, dtype=np.uint64)
    codes = _CODE[reads]
    bad = np.concatenate([[0], np.cumsum(codes == 255)])
    starts = np.arange(n - k + 1, dtype=np.int64)
    ok = bad[starts + k] == bad[starts]
    offs = offsets.astype(np.int64)
    read_of = np.searchsorted(offs, starts, side="right") - 1
    ok &= starts + k <= offs[read_of + 1]
    c = codes.astype(np.uint64)
    key = np.zeros(n - k + 1, dtype=np.uint64)
    for i in range(k):
        key = (key << np.uint64(2)) | c[i:n - k + 1 + i]
    return key[ok]


def revcomp_keys(keys: np.ndarray, k: int) -> np.ndarray:
    """Reverse complement of 2-bit keys: complement every code, reverse the
    order of the k codes."""
    x = ~keys.astype(np.uint64)
    # reverse the 32 2-bit groups of the 64-bit word, then drop the 32 - k
    # groups that came from the unused high end
    m = np.uint64
    x = ((x >> m(2)) & m(0x3333333333333333)) | ((x & m(0x3333333333333333)) << m(2))
    x = ((x >> m(4)) & m(0x0F0F0F0F0F0F0F0F)) | ((x & m(0x0F0F0F0F0F0F0F0F)) << m(4))
    x = x.byteswap()
    return x >> m(64 - 2 * k)


def strand_free(keys: np.ndarray, k: int) -> np.ndarray:
    keys = np.asarray(keys, dtype=np.uint64)
    return np.minimum(keys, revcomp_keys(keys, k))


def exact_counts(reads: np.ndarray, offsets: np.ndarray, k: int):
    """(k-mers in strand-independent form, sorted; their exact counts)."""
    return np.unique(strand_free(window_keys(reads, offsets, k), k), return_counts=True)


def compare(exact_keys, exact_cnt, distinct, trust, err, k: int, tau: int) -> dict:
    """KmerCo's lists against exact counts.  Reported k-mers always exist;
    collisions make KmerCo miss distinct k-mers (their first occurrence finds
    a counter already set) and over-count, so trustworthy recall is limited
    by the distinct recall and its precision by over-counting."""
    d = np.unique(strand_free(distinct, k))
    t = np.unique(strand_free(trust, k))
    e = np.unique(strand_free(err, k))
    true_trust = exact_keys[exact_cnt > tau]
    tp = int(np.isin(t, true_trust, assume_unique=True).sum())
    # counters never under-count, so a reported k-mer whose exact count is
    # above tau must be trustworthy
    reported_true = true_trust[np.isin(true_trust, d, assume_unique=True)]
    return {
        "exact_distinct": int(len(exact_keys)),
        "exact_trustworthy": int(len(true_trust)),
        "kmerco_distinct": int(len(distinct)),
        "kmerco_trustworthy": int(len(trust)),
        "kmerco_erroneous": int(len(err)),
        "distinct_unique": bool(len(d) == len(distinct)),
        "distinct_all_exist": bool(np.isin(d, exact_keys, assume_unique=True).all()),
        "distinct_recall": len(d) / max(1, len(exact_keys)),
        # 1.0 when nothing is claimed / nothing is to be found
        "trustworthy_precision": tp / len(t) if len(t) else 1.0,
        "trustworthy_recall": tp / len(true_trust) if len(true_trust) else 1.0,
        "split_is_partition": bool(len(t) + len(e) == len(d)
                                   and not np.isin(t, e, assume_unique=True).any()),
        "trustworthy_missed_among_reported": int(
            (~np.isin(reported_true, t, assume_unique=True)).sum()),
    }


def placement(nbytes: int) -> str:
    """Where a countBF of nbytes fits on MI355X: one XCD's L2 (4 MB), the
    eight L2s together, the 256 MB Infinity Cache, or only HBM."""
    if nbytes <= 4 << 20:
        return "L2 (one XCD)"
    if nbytes <= 32 << 20:
        return "L2 (8 XCDs)"
    if nbytes <= 256 << 20:
        return "Infinity Cache"
    return "HBM"


def evaluate(rs, sizes, steps: int = 5, alpha: int = 8, k_h: int = 1, device="cuda",
             lists: dict | None = None):
    """One result per size factor f: countBF from Eq. (1) at f x the
    workload's sizing count, timed insert + classify, lists compared with
    the exact counts.  ``lists``, when given, receives per size factor the
    host arrays that were scored: (words, distinct, trust, err)."""
    import torch

    from . import kmerco as K
    K.load_library()
    dev = torch.device(device)
    t0 = time.perf_counter()
    ex_keys, ex_cnt = exact_counts(rs.reads, rs.offsets, rs.k)
    t_exact = time.perf_counter() - t0
    reads = torch.from_numpy(rs.reads).to(dev)
    offs = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    n = rs.n_bases
    outs = [torch.empty(max(n, 1), dtype=torch.int64, device=dev) for _ in range(3)]
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    results = []
    for f in sizes:
        X, Y = K.dims(f * rs.n_items)
        bf = K.CountBF(X, Y, alpha, k_h, device=dev)
        bf.reserve(n)

        def step():
            bf.reset(stream)
            cnt.zero_()
            bf.insert_classify(reads, offs, rs.k, rs.tau, distinct=outs[0], trust=outs[1],
                               err=outs[2], n_distinct=cnt[0:1], n_windows=cnt[1:2],
                               n_trust=cnt[2:3], n_err=cnt[3:4], stream=stream)

        step()
        bf.sync()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        secs = (time.perf_counter() - t) / steps
        bf.sync()
        nd, nw, nt, ne = (int(x) for x in cnt.cpu().tolist())
        host = lambda a, m: a[:m].cpu().numpy().view(np.uint64)  # noqa: E731
        r = {"size_factor": f, "X": X, "Y": Y, "countbf_bytes": X * Y * 8,
             "placement": placement(X * Y * 8), "n_windows": nw,
             "insertions_per_s": nw / secs, "ms_per_step": secs * 1e3}
        d, t, e = host(outs[0], nd), host(outs[1], nt), host(outs[2], ne)
        r.update(compare(ex_keys, ex_cnt, d, t, e, rs.k, rs.tau))
        if lists is not None:
            lists[f] = (bf.words.cpu().numpy().view(np.uint64), d, t, e)
        r["exact_windows"] = int(ex_cnt.sum())
        r["exact_counting_s"] = t_exact
        results.append(r)
        bf.close()
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bacterial")
    ap.add_argument("--scale", type=float, default=0.1)
    ap.add_argument("--sizes", default="0.125,0.5,1,4,16")
    ap.add_argument("--steps", type=int, default=5)
    a = ap.parse_args()
    import synth
    rs = synth.config(a.workload, scale=a.scale)
    for r in evaluate(rs, [float(x) for x in a.sizes.split(",")], a.steps):
        r.update({"workload": a.workload, "scale": a.scale, "k": rs.k, "tau": rs.tau})
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
