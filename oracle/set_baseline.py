"""Host throughput of the oracle on the 256-set workload: independent sets in
parallel worker processes (the sets share nothing), for the benchmark's
batched form.  Test infrastructure like the rest of this package; run as
``python -m oracle.set_baseline --sets S --workers W`` (prints one JSON
line).  Only the first S sets are run, a bounded sample of the workload."""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import time


def _one(args):
    reads, offsets, k, tau, X, Y = args
    import oracle
    _, _, _, _, nw = oracle.run_kmerco(reads, offsets, k, tau, X, Y)
    return nw


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=64)
    ap.add_argument("--workers", type=int, default=16)
    a = ap.parse_args()
    import oracle
    from synth.reads import _cfg_batched
    oracle.build(force=False)
    sets = _cfg_batched(1.0, first=a.sets)
    jobs = []
    for rs in sets:
        X, Y = oracle.dims(rs.n_items)
        jobs.append((rs.reads, rs.offsets, rs.k, rs.tau, X, Y))
    workers = max(1, min(a.workers, os.cpu_count() or 1, len(jobs)))
    ctx = mp.get_context("fork")  # this process never touches a GPU
    t = time.perf_counter()
    with ctx.Pool(workers) as pool:
        windows = sum(pool.map(_one, jobs, chunksize=1))
    secs = time.perf_counter() - t
    print(json.dumps({"value": windows / secs, "unit": "insertions/s", "cores": workers,
                      "kind": "oracle",
                      "sample": f"first {len(jobs)} of 256 sets ({windows} k-mers), insert + "
                                f"classify per set, one single-threaded C oracle process per "
                                f"set on {workers} worker processes, {secs:.1f} s"}))


if __name__ == "__main__":
    main()
