"""KmerCo on one MI355X: k-mer insertions/s of the full hot path.

Headline (the default workload, "large"): 32 M reads of 250 bases (8 Gbases)
into an 8 GB countBF (31627 x 31657 cells), k = 31, tau = 5.  One step is
one KmerCo pass over that input with its reads already resident in HBM:
clear the countBF, then kc_insert_classify (the insertion phase: ingest,
binned counting and first-seen resolution in LDS, ordered distinct output;
the classification phase: Query-II of each distinct k-mer against the final
countBF, ordered trustworthy / erroneous split).  The metric counts one
insertion per valid k-mer window, as the paper's insertions-per-second
figure does (number of insertions / insertion time).

The same line carries, on the same input and the same countBF words, the
batched form (kc_batch_insert with the whole input as one set: tuned, then
replayed from a HIP graph), and as extra keys the bacterial workload (plain),
the 256-set workload (256 plain calls vs one batched call) and the serving
form.  Every leg is checked against the oracle's digests.

Kernel times: a few untimed steps with every kernel bracketed by HIP events
give the per-phase breakdown ("phases"); during the timed steps the library
records events around the dominant kernel only, whose average launch gives
the roofline.  "step_roofline" prices the whole step: the per-insertion
byte model of a random-access countBF insert against 8 TB/s and at the
random-access rates measured in the same run, and this design's own bound
(each phase's algorithmic bytes at the copy bandwidth measured in the same
run, plus the hashing kernel's integer operations at the VALU peak).

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
                    [--forms batched,bacterial,sets,serving|none]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# 32-bit integer VALU operations: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
ALU_PEAK_GOPS = 256 * 64 * 2.4

# Algorithmic 32-bit integer operations per valid k-mer window of the hashing
# kernel (k_h = 1), counted from the method's definitions: rolling update of
# the forward and reverse-complement keys (2 x 8), the high word of H_1 for
# both strands and the low word for the canonical one (3 MurmurHash3 x86_32
# evaluations of an 8-byte key, 23 ops each), the canonical compare/select
# (4), the slot map h mod X and h mod Y (12 each as a Barrett reduction of a
# 64-bit value), h mod eta (1 for a power-of-two eta) and w = i*Y + j (3).
OPS_PER_WINDOW = 16 + 3 * 23 + 4 + 2 * 12 + 1 + 3
# each further hash function H_a: 2 MurmurHash3 evaluations + its slot map
OPS_PER_EXTRA_HASH = 2 * 23 + 2 * 12 + 1 + 3
# k-mers of 33..64 bases: 128-bit keys (4 words) rolled for both strands
# (2 x 16), MurmurHash3 over 16 bytes (4 blocks: 37 ops), a 4-word select (6)
OPS_PER_WINDOW_WIDE = 2 * 16 + 3 * 37 + 6 + 2 * 12 + 1 + 3
OPS_PER_EXTRA_HASH_WIDE = 2 * 37 + 2 * 12 + 1 + 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["tiny", "bacterial", "large"])
    ap.add_argument("--alpha", type=int, default=8, help="counter length (bits)")
    ap.add_argument("--size", type=float, default=1.0,
                    help="countBF sized for this multiple of the workload's sizing count")
    ap.add_argument("--k-h", type=int, default=1, help="hash functions")
    ap.add_argument("--k", type=int, default=0,
                    help="k-mer length (0: the workload's own; 33..64 for two-word keys)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-reads", type=int, default=0,
                    help="reads of the oracle's sample (0: about 20 s of oracle work)")
    ap.add_argument("--cpu-sample-sets", type=int, default=64,
                    help="sets of the 256-set workload in the parallel oracle baseline")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--forms", default="batched,bacterial,sets,serving",
                    help="comma list of extra legs: batched (same input, batched form), "
                         "bacterial (plain, bacterial workload), sets (the 256-set workload, "
                         "plain vs batched), serving; or none")
    ap.add_argument("--serving-seconds", type=float, default=5.0)
    ap.add_argument("--serving-lanes", type=int, default=2)
    ap.add_argument("--form-steps", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=5,
                    help="untimed steps with every kernel timed (the per-phase breakdown); "
                         "the timed steps record events around the dominant kernel only")
    return ap.parse_args()


def sha(t) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy().view(np.uint64)).tobytes()).hexdigest()


def algorithmic_bytes(phase: str, n_bases: int, n_windows: int, n_distinct: int, k_h: int,
                      n_words: int, n_chunks: int = 1, partitioned: bool = False,
                      binned: bool = True, key_bytes: int = 8, entry_bytes=None,
                      classified=None, carried=0) -> float:
    """Bytes one step's launches of `phase` must move by their definition
    (logical accesses, not cache lines), summed over the step's launches:
    see the per-kernel table in the design notes.  classified: positions the
    insert's classification covers in the position domain (None: the
    classification of a key list)."""
    entries = n_windows * k_h
    if phase == "bin_count":         # packed input, a 4-byte slot id (+ partition byte)
        return n_bases * (0.5 + (5 if partitioned else 4) * k_h)
    if phase == "bin_part":          # slot ids + partition bytes in, 8-byte entries out
        return n_bases * 5 * k_h + entries * 8
    if phase == "part_count":        # entries of the partition lists in
        return entries * 8
    # bytes per entry: the single-level path's lists are 6-byte entries; the
    # partitioned path's partition and bucket lists are 8-byte entries and its
    # region lists 6-byte ones; the batched form's fused kernels keep 8
    ent = entry_bytes or 6
    if phase == "bin_bucket":        # slot ids (or partition-list entries) in, entries out
        return entries * 16 if partitioned else n_bases * 4 * k_h + entries * ent
    if phase == "bin_region":        # bucket-list entries in, region-list entries out
        return entries * (8 + ent) if partitioned else entries * 2 * ent
    if phase == "region":            # entries in, countBF cells read + written per chunk, flags
        b = entries * ent + n_chunks * n_words * 16 + n_distinct
        if carried:                  # carried records: 6 B written, then 2 B read + 2 B marked
            b += n_distinct * carried / n_bases * 10
        return b
    if phase == "tile_count":        # flag byte per position (+ packed input when the
        return n_bases * (1.0 if binned else 1.5)  # insert passes did not count windows)
    if phase == "claim_increment":   # cell RMW + first-seen entry RMW per slot, packed input
        return n_windows * k_h * (16 + 8) + n_bases * 0.5
    if phase == "claim":             # cell read + entry RMW per slot
        return n_windows * k_h * (8 + 8) + n_bases * 0.5
    if phase == "increment":         # cell RMW per slot
        return n_windows * k_h * 16 + n_bases * 0.5
    if phase == "resolve":           # entry read per slot, winner reset, flags
        return n_windows * k_h * 4 + n_distinct * 4 + n_bases * (0.5 + 0.125)
    if phase == "winners":           # first-seen records: two distribution passes (6 B in,
        return n_distinct * 22 + n_bases  # 4 B out, 4 B in and out), 4 B into the flag blocks,
                                          # flag bytes written in 16-byte groups
    if phase == "reset":             # the countBF's cells written (cleared)
        return n_words * 8
    if phase == "ingest":            # ASCII in, packed codes + bitmaps out, flag bytes cleared
        return n_bases * 2.5
    if phase == "valid_windows":     # invalid-base and read-start bits in, valid-window bits out
        return n_bases * 3 / 8
    if phase == "scatter":           # flag byte + packed input, keys out (distinct + split)
        return n_bases * 1.5 + n_distinct * 2 * key_bytes
    if phase == "classify_mark":
        if classified is not None:   # flag byte + packed codes per position, a cell per
            return classified * 1.25 + n_distinct * classified / n_bases * 8 * k_h  # slot
        return n_distinct * (key_bytes + 8 * k_h + 0.125)  # key + cell per slot, mask out
    if phase == "classify_scatter":  # key in, key out, mask
        return n_distinct * (2 * key_bytes + 0.125)
    return 0.0


def traffic_for(phase: str, workload: str):
    """HBM bytes per launch of a phase, from the committed rocprofv3 --pmc
    summary of this workload (FETCH_SIZE and WRITE_SIZE, calibrated on a
    copy kernel), if the kernel sources have not changed since; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    ph = rec.get("phases", {}).get(phase)
    return None if ph is None else ph.get("bytes_per_launch")


# the sources that define the kernels (host-only API code does not change
# what a kernel moves)
KERNEL_SOURCES = ["kc_batched.hip", "kc_batched.hpp", "kc_bin_hash.hpp", "kc_binned.hip", "kc_device.hpp",
                  "kc_kernels.hip", "kc_kernels.hpp", "kc_scan.hip"]


def code_text(src: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed:
    what decides the compiled code (a comment edit keeps the counters).
    String and character literals are kept whole."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_digest() -> str:
    """Digest of the kernel sources (their code, comments aside) the
    committed traffic counters belong to."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2305_07545_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(code_text(f.read()).encode())
    return h.hexdigest()


def cpu_baseline(rs, X, Y, n_sample_reads, k=0):
    """The oracle, as it is, on the first reads of the same workload with the
    same countBF dimensions, on one host core."""
    import oracle
    oracle.build(force=False)
    n = min(n_sample_reads, rs.n_reads)
    sub = rs.subset(0, n)
    t = time.perf_counter()
    _, _, _, _, nw = oracle.run_kmerco(sub.reads, sub.offsets, k or rs.k, rs.tau, X, Y)
    secs = time.perf_counter() - t
    return {"value": nw / secs, "unit": "insertions/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {rs.n_reads} reads ({nw} k-mers), insert + classify, "
                      f"countBF {X}x{Y}, single-threaded C oracle, {secs:.1f} s",
            "host": host_cpu()}


def host_cpu() -> dict:
    """The host's CPU model and logical CPU count (context for the oracle's
    timing)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def h2d_reads(rs, dev, reps: int = 3) -> dict:
    """The host-to-device copy of the workload's reads and offsets from
    pinned memory (outside the timed steps, which start from device-resident
    reads): its time, and the insertion rate a step would reach if the reads
    had to cross PCIe first."""
    import numpy as np
    import torch
    reads_h = torch.from_numpy(rs.reads).pin_memory()
    offs_h = torch.from_numpy(rs.offsets.view(np.int64)).pin_memory()
    reads_d = torch.empty_like(reads_h, device=dev)
    offs_d = torch.empty_like(offs_h, device=dev)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        reads_d.copy_(reads_h, non_blocking=True)
        offs_d.copy_(offs_h, non_blocking=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    secs = sorted(times)[len(times) // 2]
    nbytes = reads_h.numel() + offs_h.numel() * 8
    return {"ms": secs * 1e3, "bytes": nbytes, "GBps": nbytes / secs / 1e9}


def set_baseline(n_sets: int):
    """The oracle on the first sets of the 256-set workload, one process per
    set on the host's cores (the sets are independent), started as a child
    program that never touches the GPU."""
    import subprocess
    r = subprocess.run([sys.executable, "-m", "oracle.set_baseline", "--sets", str(n_sets),
                        "--workers", "16"], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def ops_per_window(k_h: int, alpha: int, k: int = 31) -> int:
    """Algorithmic integer ops per valid window: l = h mod eta is one AND
    when eta = 64 / alpha is a power of two, else a Barrett reduction
    (12 ops, like h mod X), once per hash function."""
    eta = 64 // alpha
    l_extra = 0 if eta & (eta - 1) == 0 else 11
    first, extra = (OPS_PER_WINDOW_WIDE, OPS_PER_EXTRA_HASH_WIDE) if k > 32 else \
        (OPS_PER_WINDOW, OPS_PER_EXTRA_HASH)
    return first + l_extra + (k_h - 1) * (extra + l_extra)


def roofline_of(phases, steps, n_bases, n_windows, n_distinct, k_h, n_words, workload,
                n_chunks=1, partitioned=False, alpha=8, k=31, entry_bytes=None, classified=None,
                carried=0):
    """Roofline of the phase with the largest total time: the hashing kernel
    against the integer-VALU peak (algorithmic ops per window), the others
    against HBM (algorithmic bytes), per launch over the average launch."""
    if not phases:
        return None
    dom = max(phases, key=lambda k: phases[k][0])
    avg_s = phases[dom][0] / phases[dom][1] / 1e3
    per_step = phases[dom][1] / max(1, steps)
    traffic = traffic_for(dom, workload) if k <= 32 else None
    if dom == "bin_count":
        ops = n_windows * ops_per_window(k_h, alpha, k) / per_step
        achieved = ops / avg_s / 1e9
        return {"bound": "alu", "achieved": round(achieved, 1), "peak": round(ALU_PEAK_GOPS, 1),
                "unit": "Gop/s", "frac": round(achieved / ALU_PEAK_GOPS, 4), "traffic": traffic,
                "kernel": dom, "algorithmic_ops_per_launch": ops,
                "ops_per_window": ops_per_window(k_h, alpha, k),
                "avg_launch_ms": round(avg_s * 1e3, 4), "launches_per_step": per_step}
    nbytes = algorithmic_bytes(dom, n_bases, n_windows, n_distinct, k_h, n_words, n_chunks,
                               partitioned, key_bytes=8 if k <= 32 else 16,
                               entry_bytes=entry_bytes, classified=classified,
                               carried=carried) / per_step
    achieved = nbytes / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": dom,
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": round(avg_s * 1e3, 4),
            "launches_per_step": per_step}


def hbm_rooflines(phases, steps, n_bases, n_windows, n_distinct, k_h, n_words, workload,
                  n_chunks=1, partitioned=False, k=31, classified=None, carried=0):
    """The HBM roofline of every memory-bound phase (all but the hashing)."""
    out = {}
    for ph, (ms, launches) in phases.items():
        b = algorithmic_bytes(ph, n_bases, n_windows, n_distinct, k_h, n_words, n_chunks,
                              partitioned, key_bytes=8 if k <= 32 else 16,
                              classified=classified, carried=carried)
        if ph == "bin_count" or b <= 0:
            continue
        per_step = launches / max(1, steps)
        avg_s = ms / launches / 1e3
        gbs = b / per_step / avg_s / 1e9
        out[ph] = {"achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                   "traffic": traffic_for(ph, workload) if k <= 32 else None}
    return out


def batched_leg(args, dev):
    """The 256-set workload, plain (one kc_insert_classify per set, in
    sequence on one stream) against batched (one kc_batch_insert, autotuned
    once, then replayed from a HIP graph).  Same filters, same outputs."""
    import numpy as np
    import torch

    import paper_2305_07545_amd as P
    import synth

    t_gen = time.perf_counter()
    sets = synth.config("batched")
    t_gen = time.perf_counter() - t_gen
    n = len(sets)
    # graph capture needs a non-default stream; the plain calls use it too
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        return _batched_leg(args, dev, sets, stream, t_gen)


def _batched_leg(args, dev, sets, stream, t_gen):
    import numpy as np
    import torch

    import paper_2305_07545_amd as P
    n = len(sets)
    packed, poffs, spans = P.pack_read_sets([(rs.reads, rs.offsets) for rs in sets])
    reads = torch.from_numpy(packed).to(dev)
    offs = torch.from_numpy(poffs.view(np.int64)).to(dev)
    # plain calls take each set's own buffers
    own = [(torch.from_numpy(rs.reads).to(dev), torch.from_numpy(rs.offsets.view(np.int64)).to(dev))
           for rs in sets]
    bases = [rs.n_bases for rs in sets]
    starts = np.concatenate([[0], np.cumsum(bases)]).astype(np.int64)
    total = int(starts[-1])
    out = {name: torch.empty(max(total, 1), dtype=torch.int64, device=dev)
           for name in ("distinct", "trust", "err")}
    counters = torch.zeros((n, 4), dtype=torch.int64, device=dev)
    filters, entries = [], []
    for i, (rs, (base, nb, _, _)) in enumerate(zip(sets, spans)):
        X, Y = P.dims(rs.n_items)
        f = P.CountBF(X, Y, 8, 1, device=dev)
        filters.append(f)
        sl = slice(int(starts[i]), int(starts[i + 1]))
        e = {"filter": f, "first_base": base, "n_bases": nb, "k": rs.k, "tau": rs.tau,
             "n_distinct": counters[i, 0:1], "n_windows": counters[i, 1:2],
             "n_trust": counters[i, 2:3], "n_err": counters[i, 3:4]}
        e.update({name: out[name][sl] for name in out})
        entries.append(e)

    def plain_step():
        counters.zero_()
        for e, (r, o) in zip(entries, own):
            e["filter"].reset(stream)
            e["filter"].insert_classify(r, o, e["k"], e["tau"], distinct=e["distinct"],
                                        trust=e["trust"], err=e["err"],
                                        n_distinct=e["n_distinct"], n_windows=e["n_windows"],
                                        n_trust=e["n_trust"], n_err=e["n_err"], stream=stream)

    batch = P.Batch()

    def batch_step(tune=False):
        counters.zero_()
        batch.insert(entries, reads, offs, reset=True, graph=not tune, tune=tune, stream=stream)

    def timed(step, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def check():
        import json as _json
        ref_path = os.path.join(ROOT, "tests", "golden", "batched_digests.json")
        if args.no_verify or not os.path.exists(ref_path):
            return None
        ref = _json.load(open(ref_path))["sets"]
        c = counters.cpu().numpy()
        for i, (e, r) in enumerate(zip(entries, ref)):
            nd, nw, nt, ne = (int(x) for x in c[i])
            if (nd, nw, nt, ne) != (r["n_distinct"], r["n_windows"], r["n_trust"], r["n_err"]):
                return False
            if (sha(e["filter"].words) != r["words_sha256"]
                    or sha(e["distinct"][:nd]) != r["distinct_sha256"]
                    or sha(e["trust"][:nt]) != r["trust_sha256"]
                    or sha(e["err"][:ne]) != r["err_sha256"]):
                return False
        return True

    steps = max(1, args.form_steps)
    plain_step()
    plain_step()
    plain_s = timed(plain_step, steps)
    plain_ok = check()
    for f in filters:
        f.sync()
    n_windows = int(counters[:, 1].sum().item())

    batch_step(tune=True)
    batch_step()
    batch_step()
    batch_s = timed(batch_step, steps)
    batch.sync()
    batch_ok = check()
    # per-phase times come from eager launches (events are not recorded
    # inside graph replays)
    batch.profile(True)
    eager_s = timed(lambda: batch.insert(entries, reads, offs, reset=True, stream=stream), steps)
    phases = batch.profile_read()
    batch.profile(False)
    batch.sync()
    n_distinct = int(counters[:, 0].sum().item())
    n_words = sum(int(f.layout.X) * int(f.layout.Y) for f in filters)
    res = {
        "workload": "batched: 256 read sets, own countBF each",
        "n_sets": n, "n_reads": sum(rs.n_reads for rs in sets), "n_bases": total,
        "n_windows": n_windows, "n_distinct": n_distinct,
        "countbf_bytes_total": n_words * 8,
        "value": n_windows / batch_s, "plain_value": n_windows / plain_s,
        "unit": "insertions/s", "speedup_vs_plain": plain_s / batch_s,
        "ms_per_step": batch_s * 1e3, "plain_ms_per_step": plain_s * 1e3,
        "eager_ms_per_step": eager_s * 1e3,
        "steps": steps, "tile": batch.tile, "graph": True,
        "verified_vs_oracle_digests": {"batched": batch_ok, "plain": plain_ok},
        "phases": {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in phases.items()},
        "roofline": roofline_of(phases, steps, total, n_windows, n_distinct, 1, n_words,
                                "batched", entry_bytes=8),
        "tuned": {"work_item_positions": batch.tile},
        "input_generation_s": round(t_gen, 1),
    }
    for f in filters:
        f.close()
    batch.close()
    return res


def serving_digests_ok(args, w, server, sessions, dims, res, outs):
    """The paced run against the oracle's digests of the serving trace: every
    request's counts, every session's final words and distinct list, and
    each session's last classification (its outputs are the last written to
    the session's lists).  None without digests for this trace."""
    import hashlib

    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "serving_digests.json")
    if args.no_verify or not os.path.exists(path):
        return None
    ref = json.load(open(path))
    if ref["duration_s"] != args.serving_seconds or ref["n_requests"] != len(w.requests):
        return None

    def h(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()

    try:
        for s in ref["sessions"]:
            g = s["session"]
            X, Y = dims[g]
            if (s["X"], s["Y"], s["k"]) != (X, Y, w.ks[g]):
                return False
            for r in s["requests"]:
                got = res[r["request"]]
                if (got["n_windows"], got["n_new"]) != (r["n_windows"], r["n_new"]):
                    return False
                if "n_trust" in r and (got["n_trust"], got["n_err"]) != (r["n_trust"],
                                                                         r["n_err"]):
                    return False
            if h(server.read_words(sessions[g], X * Y)) != s["words_sha256"]:
                return False
            if h(server.read_distinct(sessions[g], 0, s["n_distinct"])) != s["distinct_sha256"]:
                return False
            lc = s["last_classify"]
            if lc:
                nt, ne = res[lc["request"]]["n_trust"], res[lc["request"]]["n_err"]
                if h(outs[g][0][:nt].cpu().numpy().view(np.uint64)) != lc["trust_sha256"] or \
                        h(outs[g][1][:ne].cpu().numpy().view(np.uint64)) != lc["err_sha256"]:
                    return False
    except Exception:  # a list shorter than the oracle's cannot be read that far
        return False
    return True


def serving_leg(args, dev):
    """The serving trace replayed in real time: Poisson arrivals (50/s) of
    insert / insert+classify requests on 16 device-resident sessions under a
    200 GB budget.  Latency = completion - submission on the server clock;
    throughput = k-mers inserted / (last completion - first submission)."""
    import math

    import numpy as np
    import torch

    import paper_2305_07545_amd as P
    from paper_2305_07545_amd import serve
    import synth

    t_gen = time.perf_counter()
    w = synth.serving_workload(duration_s=args.serving_seconds)
    n = len(w.requests)
    # pinned host copies: the requests' reads are runs of these pools
    pools = [torch.from_numpy(r).pin_memory() for r, _ in w.pools]
    n_off = sum(q.n_reads + 1 for q in w.requests)
    offs_all = torch.empty(n_off, dtype=torch.int64).pin_memory()
    bufs, pos, expect_windows = [], 0, 0
    for i, q in enumerate(w.requests):
        _, o = w.request_reads(i)
        lo = int(w.pools[q.genome][1][q.first_read])
        view = offs_all[pos:pos + len(o)]
        view.copy_(torch.from_numpy(o.view(np.int64)))
        bufs.append((pools[q.genome][lo:lo + int(o[-1])], view))
        pos += len(o)
        lens = np.diff(o.astype(np.int64))
        expect_windows += int(np.maximum(lens - w.ks[q.genome] + 1, 0).sum())
    t_gen = time.perf_counter() - t_gen

    budget = 200 * 10**9
    server = P.Server(memory_budget=budget,
                      lane_bases=max(w.request_bases(i) for i in range(n)),
                      lane_reads=max(q.n_reads for q in w.requests), lane_requests=64,
                      lanes=args.serving_lanes)
    caps = [int(math.ceil(1.2 * d)) + 4096 for d in w.expected_distinct]
    dims = [P.dims(x) for x in w.n_items]
    sessions = [server.open(X, Y, w.ks[g], caps[g]) for g, (X, Y) in enumerate(dims)]
    outs = [(torch.empty(c, dtype=torch.int64, device=dev), torch.empty(c, dtype=torch.int64,
                                                                         device=dev))
            for c in caps]

    def submit(i):
        q = w.requests[i]
        reads, offs = bufs[i]
        kw = {}
        if q.classify:
            kw = {"classify": True, "tau": q.tau, "trust": outs[q.genome][0],
                  "err": outs[q.genome][1]}
        return server.submit(sessions[q.genome], reads, offs, **kw)

    res = serve.replay(server, [q.t for q in w.requests], submit)
    st = server.stats()
    verified = serving_digests_ok(args, w, server, sessions, dims, res, outs)
    server.close_server()

    # capacity: the same requests all submitted at once to fresh sessions
    sat = P.Server(memory_budget=budget,
                   lane_bases=max(w.request_bases(i) for i in range(n)),
                   lane_reads=max(q.n_reads for q in w.requests), lane_requests=64,
                   lanes=args.serving_lanes)
    server = sat  # submit() now targets the fresh server and its sessions
    sessions[:] = [sat.open(X, Y, w.ks[g], caps[g]) for g, (X, Y) in enumerate(dims)]
    res_sat = serve.replay(sat, [0.0] * n, submit)
    sat_span = max(r["t_done"] for r in res_sat) - min(r["t_submit"] for r in res_sat)
    sat_ok = [r["n_windows"] for r in res_sat] == [r["n_windows"] for r in res] and \
        [r["n_new"] for r in res_sat] == [r["n_new"] for r in res] and \
        all(r["status"] == 0 for r in res_sat)
    sat_st = sat.stats()
    ok = all(r["status"] == 0 for r in res)
    windows = sum(r["n_windows"] for r in res)
    nxt = [0] * len(sessions)
    for i, q in enumerate(w.requests):  # each request continues its session's list
        ok &= res[i]["distinct_first"] == nxt[q.genome]
        nxt[q.genome] += res[i]["n_new"]
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    out = {
        "workload": "serving: 16 sessions, Poisson 50 req/s, 10k-2M reads per request",
        "requests": n, "duration_s": args.serving_seconds,
        "classify_requests": sum(q.classify for q in w.requests),
        "n_bases": sum(w.request_bases(i) for i in range(n)),
        "n_windows": windows, "value": windows / span, "unit": "insertions/s",
        "latency": serve.latency_summary(res),
        "checks": {"statuses_ok_and_lists_contiguous": bool(ok),
                   "windows_equal_sum_of_L_minus_k_plus_1": windows == expect_windows},
        "verified_vs_oracle_digests": verified,
        "memory_budget_bytes": budget, "session_bytes": st["session_bytes"],
        "staging_bytes": st["staging_bytes"], "batches": st["batches"],
        "batched_requests": st["batched_requests"], "plain_requests": st["plain_requests"],
        "max_batch": st["max_batch"], "lanes": args.serving_lanes,
        "lanes_in_flight_max": st["lanes_in_flight_max"],
        "saturated": {"value": windows / sat_span, "unit": "insertions/s",
                      "makespan_s": sat_span, "latency": serve.latency_summary(res_sat),
                      "batches": sat_st["batches"], "max_batch": sat_st["max_batch"],
                      "lanes_in_flight_max": sat_st["lanes_in_flight_max"],
                      "same_counts_as_paced_run": bool(sat_ok)},
        "countbf_bytes": [X * Y * 8 for X, Y in dims],
        "input_generation_s": round(t_gen, 1),
    }
    sat.close_server()
    return out


# per-workload oracle sample (reads) of about 10-30 s of single-core work
CPU_SAMPLE_READS = {"tiny": 10_000, "bacterial": 300_000, "large": 200_000}


def copy_bandwidth(dev, nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Bytes moved per second (read + write) by a device-to-device copy of
    nbytes: the streaming rate this part reaches, measured in this run."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    return 2 * nbytes / best


def random_read_rate(words, n: int = 1 << 26, reps: int = 3) -> float:
    """8-byte reads per second at uniformly random positions of `words` (a
    gather over the countBF's own footprint, measured in this run)."""
    import torch
    g = torch.Generator(device=words.device)
    g.manual_seed(7)
    idx = torch.randint(0, words.numel(), (n,), device=words.device, generator=g)
    out = torch.empty(n, dtype=words.dtype, device=words.device)
    torch.index_select(words, 0, idx, out=out)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.index_select(words, 0, idx, out=out)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del idx, out
    return n / best


def random_access_rates(footprint: int, ops: int = 1 << 27) -> dict:
    """Uniform-random operations per second over a buffer of the countBF's
    size, measured in this run by the library's microbenchmarks: 64-bit
    load + compare-and-swap increments (a saturating counter update), 8-byte
    reads and 32-bit atomicMin (a first-seen claim)."""
    from paper_2305_07545_amd import microbench as mb
    return {"rmw64_per_s": mb.rate("cas64", footprint, ops),
            "read64_per_s": mb.rate("read64", footprint, ops),
            "min32_per_s": mb.rate("min32", footprint, ops)}


def classified_positions(plan, n_bases, k_h):
    """Positions an insert's classification rereads against the final
    countBF: with one hash function the binned paths' last region pass marks
    the k-mers first seen in the last chunk, and with the carried
    classification those of the earlier chunks too (none are reread);
    otherwise the earlier chunks' positions are classified afterwards, and
    every position with several hash functions or on the direct path."""
    if plan["path"] != "direct" and k_h == 1:
        return 0 if plan.get("carried") else (plan["n_chunks"] - 1) * plan["chunk"]
    return n_bases


def carried_positions(plan):
    """Positions whose first-seen records the carried classification keeps
    (the chunks before the last)."""
    return (plan["n_chunks"] - 1) * plan["chunk"] if plan.get("carried") else 0


def step_roofline(phases, steps, n_bases, n_windows, n_distinct, k_h, n_words, n_chunks,
                  partitioned, alpha, k, ms_per_step, copy_Bps, rand_rate, classified,
                  carried=0, rates=None):
    """The whole step against three bounds.
    random_access_model: the per-insertion byte model of a countBF insert (k_h
    random 64-bit read-modify-writes of 16 B, one 8 B pre-chunk counter read
    for first-seen, 16 B per new k-mer for its claim and its key, the input
    bytes per insertion and 1/8 B of flags) at the nominal 8 TB/s.
    random_access_model_measured_rates: the time the same operations take at the
    uniform-random update, read and claim rates measured over the countBF's
    footprint in this run (frac = that time / the measured step: above 1
    when the step beats a random-access implementation of the operations).
    design_bound: this design's own floor, each phase's algorithmic bytes at
    the copy bandwidth measured in this run, the hashing kernel's integer
    operations at the VALU peak, and the classification's random countBF
    reads at the random-read rate measured over the countBF in this run (for
    the classified share of the positions: distinct k-mers counted as spread
    evenly over the positions, which front-loaded first occurrences make an
    underestimate of the bound)."""
    secs = ms_per_step / 1e3
    f_new = n_distinct / max(1, n_windows)
    b_ins = 16 * k_h + 8 + 16 * f_new + n_bases / max(1, n_windows) + 0.125
    achieved = n_windows * b_ins / secs / 1e9
    kb = 8 if k <= 32 else 16
    per_phase = {}
    for ph in phases:
        if ph == "bin_count":
            t = n_windows * ops_per_window(k_h, alpha, k) / (ALU_PEAK_GOPS * 1e9)
        elif ph == "classify_mark":
            share = classified / max(1, n_bases)
            t = share * n_distinct * k_h / rand_rate + classified * 1.25 / copy_Bps
        else:
            t = algorithmic_bytes(ph, n_bases, n_windows, n_distinct, k_h, n_words, n_chunks,
                                  partitioned, key_bytes=kb, carried=carried) / copy_Bps
        per_phase[ph] = round(t * 1e3, 3)
    bound_ms = sum(per_phase.values())
    measured = None
    if rates:
        # the model's per-insertion operations at the random-access rates
        # measured over the countBF's footprint: a saturating 64-bit update
        # per hash function, the pre-chunk counter read of first-seen, a
        # 32-bit claim and its check read per new k-mer, and the streamed
        # input, keys and flags at the copy rate
        t = (n_windows * k_h / rates["rmw64_per_s"] + n_windows / rates["read64_per_s"] +
             n_distinct * (1 / rates["min32_per_s"] + 1 / rates["read64_per_s"]) +
             (n_bases + 8 * n_distinct + n_windows / 8) / copy_Bps)
        measured = {"allowed_ms": round(t * 1e3, 3), "measured_ms": round(ms_per_step, 3),
                    "frac": round(t * 1e3 / ms_per_step, 4),
                    "rates": {k_: round(v / 1e9, 2) for k_, v in rates.items()},
                    "rates_unit": "G ops/s"}
    return {
        "random_access_model": {"bytes_per_insertion": round(b_ins, 3),
                         "achieved_GBps": round(achieved, 1), "peak_GBps": HBM_PEAK_GBS,
                         "frac": round(achieved / HBM_PEAK_GBS, 4)},
        "random_access_model_measured_rates": measured,
        "design_bound": {"bound_ms": round(bound_ms, 3), "measured_ms": round(ms_per_step, 3),
                         "frac": round(bound_ms / ms_per_step, 4),
                         "copy_GBps_measured": round(copy_Bps / 1e9, 1),
                         "random_8B_reads_per_s_measured": round(rand_rate / 1e9, 2) * 1e9,
                         "valu_peak_Gops": round(ALU_PEAK_GOPS, 1),
                         "per_phase_bound_ms": per_phase},
    }


def digests_ok(ref, X, Y, k, words, lists, counts, w) -> bool:
    """The outputs against the oracle's digests of this workload and layout."""
    nd, nw, nt, ne = counts
    distinct, trust, err = lists
    return (ref["X"] == X and ref["Y"] == Y and ref["k"] == k and ref["n_windows"] == nw
            and ref["n_distinct"] == nd and ref["n_trust"] == nt and ref["n_err"] == ne
            and sha(words) == ref["words_sha256"]
            and sha(distinct[:nd * w]) == ref["distinct_sha256"]
            and sha(trust[:nt * w]) == ref["trust_sha256"]
            and sha(err[:ne * w]) == ref["err_sha256"])


def load_digests(args, workload, k, rs_k):
    if args.no_verify or (args.alpha, args.k_h, args.size) != (8, 1, 1.0):
        return None  # the digests' layout only
    name = workload if k == rs_k else f"{workload}_k{k}"
    path = os.path.join(ROOT, "tests", "golden", f"{name}_digests.json")
    return json.load(open(path)) if os.path.exists(path) else None


def plain_leg(args, dev, workload, steps, warmup, profile_steps, keep=False, extras=True):
    """The plain call on one workload: timed steps of kc_reset +
    kc_insert_classify, the per-phase breakdown, the dominant kernel's
    roofline, the whole step's roofline and the digest check."""
    import numpy as np
    import torch

    import paper_2305_07545_amd as P
    import synth

    t_gen = time.perf_counter()
    rs = synth.config(workload)
    t_gen = time.perf_counter() - t_gen
    X, Y = P.dims(rs.n_items * args.size)
    k_h, alpha = args.k_h, args.alpha
    k = args.k or rs.k
    w = P.key_words(k)
    reads = torch.from_numpy(rs.reads).to(dev)
    offs = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    n_bases = rs.n_bases
    words = torch.empty(X * Y, dtype=torch.int64, device=dev)
    bf = P.CountBF(X, Y, alpha, k_h, words=words, device=dev)
    bf.reserve(n_bases)
    plan = bf.plan(n_bases)
    stream = torch.cuda.current_stream()
    counters = torch.zeros(4, dtype=torch.int64, device=dev)  # distinct, windows, trust, err
    nd_, nw_, nt_, ne_ = (counters[i:i + 1] for i in range(4))

    # list capacities from a first pass with room for one key: the distinct
    # count reports what the list needs (the overflow is sticky, read by
    # sync), and the trustworthy and erroneous lists split it
    one = [torch.empty(w, dtype=torch.int64, device=dev) for _ in range(3)]
    bf.insert_classify(reads, offs, k, rs.tau, distinct=one[0], trust=one[1], err=one[2],
                       n_distinct=nd_, n_windows=nw_, n_trust=nt_, n_err=ne_, stream=stream)
    try:
        bf.sync()
    except P.KmercoError as e:
        if e.status != P.KC_ERANGE:
            raise
    need = int(counters[0].item())
    room = need + need // 64 + 4096
    distinct, trust, err = (torch.empty(room * w, dtype=torch.int64, device=dev)
                            for _ in range(3))
    del one

    def step():
        bf.reset(stream)
        counters.zero_()
        bf.insert_classify(reads, offs, k, rs.tau, distinct=distinct, trust=trust, err=err,
                           n_distinct=nd_, n_windows=nw_, n_trust=nt_, n_err=ne_, stream=stream)

    for _ in range(warmup):
        step()
    bf.sync()
    torch.cuda.synchronize()
    # per-phase breakdown: every kernel bracketed by events, untimed steps
    bf.profile(True)
    for _ in range(profile_steps):
        step()
    phases = bf.profile_read()
    bf.profile(False)
    dom = max(phases, key=lambda p: phases[p][0])
    # timed steps: events around the dominant kernel only (its roofline)
    bf.profile(True, phases=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = bf.profile_read()
    bf.profile(False)
    bf.sync()
    counts = [int(x) for x in counters.cpu().tolist()]
    n_distinct, n_windows, n_trust, n_err = counts
    ref = load_digests(args, workload, k, rs.k)
    verified = None if ref is None else digests_ok(
        ref, X, Y, k, words, (distinct, trust, err), counts, w)
    ms_step = elapsed * 1e3 / steps
    partitioned = plan["path"] == "partitioned"
    n_chunks = plan["n_chunks"]
    classified = classified_positions(plan, n_bases, k_h)
    carried = carried_positions(plan)
    per_phase = {p: {"avg_ms": v[0] / v[1], "launches": v[1]} for p, v in phases.items()}
    per_phase[dom]["timed_avg_ms"] = timed[dom][0] / timed[dom][1]
    roofline = roofline_of(timed, steps, n_bases, n_windows, n_distinct, k_h, X * Y, workload,
                           n_chunks, partitioned, alpha, k, classified=classified,
                           carried=carried)
    copy_Bps = copy_bandwidth(dev)
    rand = random_read_rate(words)
    rates = random_access_rates(X * Y * 8)
    out = {
        "value": n_windows * steps / elapsed, "unit": "insertions/s", "ms_per_step": ms_step,
        "steps": steps, "warmup": warmup,
        "config": {"workload": workload, "n_reads": rs.n_reads, "n_bases": n_bases, "k": k,
                   "tau": rs.tau, "X": X, "Y": Y, "alpha": alpha, "k_h": k_h,
                   "countbf_bytes": X * Y * 8, "n_windows": n_windows,
                   "n_distinct": n_distinct, "n_trust": n_trust, "n_err": n_err,
                   "plan": plan, "parallelism": "single GPU"},
        "verified_vs_oracle_digests": verified,
        "phases": per_phase,
        "phases_profiled_steps": profile_steps,
        "roofline": roofline,
        "step_roofline": step_roofline(phases_per_step(phases, profile_steps), 1, n_bases,
                                       n_windows, n_distinct, k_h, X * Y, n_chunks, partitioned,
                                       alpha, k, ms_step, copy_Bps, rand, classified,
                                       carried, rates),
        "hbm_rooflines": hbm_rooflines(phases, profile_steps, n_bases, n_windows, n_distinct,
                                       k_h, X * Y, workload, n_chunks, partitioned, k,
                                       classified, carried),
        "input_generation_s": round(t_gen, 1),
    }
    if extras:
        # classification on its own (kc_classify, Query-II over the step's
        # distinct list): within the timed steps it is fused into the region
        # pass when the insert is one chunk
        cls_ms = []
        n_keys = torch.tensor([n_distinct], dtype=torch.int64, device=dev)
        cls_out = [torch.empty(max(1, n_distinct) * w, dtype=torch.int64, device=dev)
                   for _ in range(2)]
        for _ in range(4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            bf.classify(distinct, n_keys, rs.tau, trust=cls_out[0], err=cls_out[1],
                        keys_cap=n_distinct, stream=stream)
            torch.cuda.synchronize()
            cls_ms.append((time.perf_counter() - t) * 1e3)
        bf.sync()
        med = sorted(cls_ms[1:])[1]
        out["classify_separately"] = {"ms": med, "keys": n_distinct,
                                      "keys_per_s": n_distinct / (med / 1e3)}
        del cls_out
        h2d = h2d_reads(rs, dev)
        h2d["insertions_per_s_incl_h2d"] = n_windows / ((h2d["ms"] + ms_step) / 1e3)
        out["h2d_reads"] = h2d
    bf.close()
    ctx = {"rs": rs}
    if keep:
        ctx.update({"reads": reads, "offs": offs, "words": words, "X": X, "Y": Y, "k": k,
                    "w": w, "lists": (distinct, trust, err), "counters": counters, "ref": ref,
                    "plain_ms": ms_step})
    else:
        del reads, offs, words, distinct, trust, err
    torch.cuda.empty_cache()
    return out, ctx


def phases_per_step(phases, steps):
    """{phase: (ms, launches)} totals over `steps` steps -> per step."""
    return {p: (v[0] / steps, v[1] / steps) for p, v in phases.items()}


def batched_same_input(args, dev, ctx, steps, warmup):
    """The batched form on the headline's input and countBF words: one
    kc_batch_insert call with the whole input as one set, tuned once, then
    captured into a HIP graph and replayed; outputs against the digests."""
    import torch

    import paper_2305_07545_amd as P
    rs, X, Y, k, w = ctx["rs"], ctx["X"], ctx["Y"], ctx["k"], ctx["w"]
    distinct, trust, err = ctx["lists"]
    counters = ctx["counters"]
    n_bases = rs.n_bases
    f = P.CountBF(X, Y, args.alpha, args.k_h, words=ctx["words"], device=dev)
    entry = {"filter": f, "first_base": 0, "n_bases": n_bases, "k": k, "tau": rs.tau,
             "distinct": distinct, "n_distinct": counters[0:1], "n_windows": counters[1:2],
             "trust": trust, "n_trust": counters[2:3], "err": err, "n_err": counters[3:4]}
    batch = P.Batch()
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        t = time.perf_counter()
        batch.insert([entry], ctx["reads"], ctx["offs"], reset=True, tune=True, stream=stream)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t
        for _ in range(max(1, warmup)):  # the first call captures the graph
            batch.insert([entry], ctx["reads"], ctx["offs"], reset=True, graph=True,
                         stream=stream)
        batch.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.insert([entry], ctx["reads"], ctx["offs"], reset=True, graph=True,
                         stream=stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        batch.sync()
        f.sync()
        counts = [int(x) for x in counters.cpu().tolist()]
        verified = None if ctx["ref"] is None else digests_ok(
            ctx["ref"], X, Y, k, ctx["words"], ctx["lists"], counts, w)
        # per-phase times from eager launches (events are not recorded
        # inside graph replays)
        batch.profile(True)
        for _ in range(2):
            batch.insert([entry], ctx["reads"], ctx["offs"], reset=True, stream=stream)
        phases = batch.profile_read()
        batch.profile(False)
        batch.sync()
    ms = elapsed * 1e3 / steps
    res = {
        "workload": "the headline's input as one set of kc_batch_insert, same countBF words",
        "value": counts[1] * steps / elapsed, "unit": "insertions/s", "ms_per_step": ms,
        "steps": steps, "graph": True, "speedup_vs_plain": ctx["plain_ms"] / ms,
        "tuned": {"plan": f.plan(n_bases), "work_item_positions": batch.tile,
                  "tune_s": round(tune_s, 2)},
        "verified_vs_oracle_digests": verified,
        "phases": {p: {"avg_ms": v[0] / v[1], "launches": v[1]} for p, v in phases.items()},
    }
    f.close()
    batch.close()
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU only; "
                          "--gpus must be 1 (no multi-GPU path is implemented)"}), flush=True)
        sys.exit(2)

    import torch

    import paper_2305_07545_amd as P

    P.load_library()  # fails loudly when the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    forms = [f for f in args.forms.split(",") if f and f != "none"]

    head, ctx = plain_leg(args, dev, args.workload, args.steps, args.warmup,
                          args.profile_steps, keep="batched" in forms)
    out = {
        "metric": "k-mer insertions/s",
        "value": head["value"],
        "unit": "insertions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
    }
    out.update({k: v for k, v in head.items() if k not in out})
    rs_head = ctx.pop("rs")
    if "batched" in forms:
        out["batched"] = batched_same_input(args, dev, dict(ctx, rs=rs_head),
                                            max(1, args.form_steps), max(1, args.warmup // 2))
    del ctx
    torch.cuda.empty_cache()
    if "bacterial" in forms and args.workload != "bacterial":
        leg, _ = plain_leg(args, dev, "bacterial", args.steps, args.warmup, 2, extras=False)
        out["bacterial"] = {k: leg[k] for k in ("value", "unit", "ms_per_step", "config",
                                                "verified_vs_oracle_digests", "roofline",
                                                "step_roofline", "phases")}
    if "sets" in forms:
        out["sets"] = batched_leg(args, dev)
        if not args.no_cpu_baseline:
            out["sets"]["cpu_baseline"] = set_baseline(args.cpu_sample_sets)
    if "serving" in forms:
        out["serving"] = serving_leg(args, dev)
    if not args.no_cpu_baseline:
        import synth
        rs = rs_head or synth.config(args.workload)
        n = args.cpu_sample_reads or CPU_SAMPLE_READS[args.workload]
        out["cpu_baseline"] = cpu_baseline(rs, out["config"]["X"], out["config"]["Y"], n,
                                           out["config"]["k"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
