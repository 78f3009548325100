"""Write SHA-256 digests of the oracle's outputs on the full-size workloads.

Calls only ``oracle`` and ``synth``; the GPU parity tests compare the HIP
path's outputs against these stored digests.  Usage:

    python tests/golden/make_digests.py tiny bacterial batched bacterial_k55
    python tests/golden/make_digests.py fullchunk_4201x4211 fullchunk_2621x2657 fullchunk_5801x5807
    python tests/golden/make_digests.py serving

The batched workload (256 independent read sets, each with its own countBF)
is stored set by set; its sets run in parallel host processes.  The serving
trace (16 sessions, 247 requests) is stored session by session: each
session's requests in submission order (a request inserts its reads into
its session's countBF, and a classify request then splits the session's
whole distinct list at its tau), per request the k-mers inserted, the
first-seen k-mers added and the classification's counts, per session the
final countBF words, the distinct list and its last classification; the
sessions run in parallel host processes.
"""
import hashlib
import json
import multiprocessing
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()


def digests(name: str, scale: float = 1.0, k: int = 0) -> dict:
    """k: the workload's own k when 0, else that k-mer length on its reads
    (keys of k > 32 are digested as (low, high) word pairs)."""
    rs = synth.config(name, scale)
    k = k or rs.k
    X, Y = oracle.dims(rs.n_items, 0.001)
    t = time.time()
    words, distinct, trust, err, nw = oracle.run_kmerco(rs.reads, rs.offsets, k, rs.tau, X, Y)
    secs = time.time() - t
    return {
        "workload": name, "scale": scale, "k": k, "tau": rs.tau, "X": X, "Y": Y,
        "alpha": 8, "k_h": 1, "n_reads": rs.n_reads, "n_bases": rs.n_bases,
        "n_windows": nw, "n_distinct": len(distinct), "n_trust": len(trust), "n_err": len(err),
        "words_sha256": sha(words), "distinct_sha256": sha(distinct),
        "trust_sha256": sha(trust), "err_sha256": sha(err),
        "oracle_seconds": round(secs, 2),
    }


# seeded inputs of the parity tests that are not workloads: name ->
# (read-set builder, X, Y)
def _full_chunk_reads():
    """About 280 M bases of random reads: one full binned chunk (2^28
    positions) and a tail."""
    return synth.random_reads(1500, 1_400_000, 150, 250, k=31, p_n=0.0005, tau=3)


INPUTS = {
    "fullchunk_4201x4211": (_full_chunk_reads, 4201, 4211),
    "fullchunk_2621x2657": (_full_chunk_reads, 2621, 2657),
    # a countBF of 16,448 regions (269 MB): the partitioned path
    "fullchunk_5801x5807": (_full_chunk_reads, 5801, 5807),
}


def input_digests(name: str) -> dict:
    build, X, Y = INPUTS[name]
    rs = build()
    t = time.time()
    words, distinct, trust, err, nw = oracle.run_kmerco(rs.reads, rs.offsets, rs.k, rs.tau, X, Y)
    secs = time.time() - t
    return {
        "input": name, "k": rs.k, "tau": rs.tau, "X": X, "Y": Y, "alpha": 8, "k_h": 1,
        "n_reads": rs.n_reads, "n_bases": rs.n_bases,
        "n_windows": nw, "n_distinct": len(distinct), "n_trust": len(trust), "n_err": len(err),
        "words_sha256": sha(words), "distinct_sha256": sha(distinct),
        "trust_sha256": sha(trust), "err_sha256": sha(err),
        "oracle_seconds": round(secs, 2),
    }


_SETS = []


def _one_set(i: int) -> dict:
    rs = _SETS[i]
    X, Y = oracle.dims(rs.n_items, 0.001)
    words, distinct, trust, err, nw = oracle.run_kmerco(rs.reads, rs.offsets, rs.k, rs.tau, X, Y)
    return {"set": i, "k": rs.k, "tau": rs.tau, "X": X, "Y": Y, "n_reads": rs.n_reads,
            "n_bases": rs.n_bases, "n_windows": nw, "n_distinct": len(distinct),
            "n_trust": len(trust), "n_err": len(err), "words_sha256": sha(words),
            "distinct_sha256": sha(distinct), "trust_sha256": sha(trust),
            "err_sha256": sha(err)}


def batched_digests(scale: float = 1.0, workers: int = 8) -> dict:
    _SETS[:] = synth.config("batched", scale)
    t = time.time()
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        per_set = pool.map(_one_set, range(len(_SETS)), chunksize=1)
    return {"workload": "batched", "scale": scale, "alpha": 8, "k_h": 1,
            "n_sets": len(per_set), "n_windows": sum(d["n_windows"] for d in per_set),
            "oracle_seconds_wall": round(time.time() - t, 2), "oracle_processes": workers,
            "sets": per_set}


_SERVING = []


def _serving_session(g: int) -> dict:
    w = _SERVING[0]
    X, Y = oracle.dims(w.n_items[g], 0.001)
    k = w.ks[g]
    bf = oracle.CountBF(X, Y)
    reqs, lists, last = [], [], None
    for i, q in enumerate(w.requests):
        if q.genome != g:
            continue
        reads, offs = w.request_reads(i)
        d, nw = bf.insert(reads, offs, k)
        lists.append(d)
        r = {"request": i, "n_windows": nw, "n_new": len(d)}
        if q.classify:
            t, e = bf.classify(np.concatenate(lists), q.tau)
            r.update({"tau": q.tau, "n_trust": len(t), "n_err": len(e)})
            last = {"request": i, "trust_sha256": sha(t), "err_sha256": sha(e)}
        reqs.append(r)
    distinct = np.concatenate(lists) if lists else np.zeros(0, dtype=np.uint64)
    return {"session": g, "k": k, "X": X, "Y": Y, "n_distinct": len(distinct),
            "words_sha256": sha(bf.words), "distinct_sha256": sha(distinct),
            "last_classify": last, "requests": reqs}


def serving_digests(duration_s: float = 5.0, workers: int = 8) -> dict:
    w = synth.serving_workload(duration_s=duration_s)
    _SERVING[:] = [w]
    vol = [0] * len(w.ks)
    for i, q in enumerate(w.requests):
        vol[q.genome] += w.request_bases(i)
    order = sorted(range(len(w.ks)), key=lambda g: -vol[g])  # largest first
    t = time.time()
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        done = pool.map(_serving_session, order, chunksize=1)
    sessions = sorted(done, key=lambda d: d["session"])
    return {"workload": "serving", "duration_s": duration_s, "alpha": 8, "k_h": 1,
            "n_requests": len(w.requests), "n_bases": sum(vol),
            "n_windows": sum(r["n_windows"] for s in sessions for r in s["requests"]),
            "oracle_seconds_wall": round(time.time() - t, 2), "oracle_processes": workers,
            "sessions": sessions}


if __name__ == "__main__":
    oracle.build(force=False)
    # names: tiny, bacterial, batched, large, or <workload>_k<k> (another k)
    for name in sys.argv[1:] or ["tiny", "bacterial"]:
        base, _, kk = name.partition("_k")
        if name == "batched":
            d = batched_digests()
        elif name == "serving":
            d = serving_digests()
        elif name in INPUTS:
            d = input_digests(name)
        else:
            d = digests(base, k=int(kk or 0))
        path = os.path.join(HERE, f"{name}_digests.json")
        with open(path, "w") as f:
            json.dump(d, f, indent=1)
        print(path, {k: v for k, v in d.items() if k not in ("sets", "sessions")})
