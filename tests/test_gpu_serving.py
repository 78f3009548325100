"""Serving form: every request's outputs (k-mers inserted, the first-seen
k-mers it added to its session, its classification) are the same when the
request is served alone and when it shares batches with the live mix, and
both equal the oracle run request by request on each session."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2305_07545_amd")
from paper_2305_07545_amd import serve  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    P.load_library()


@pytest.fixture(scope="module")
def workload():
    return synth.serving_workload(scale=0.005, duration_s=1.5)


def caps(w):
    return [int(math.ceil(1.5 * d)) + 1024 for d in w.expected_distinct]


class Client:
    """Host buffers, sessions and classify outputs for one run of a trace."""

    def __init__(self, server, w, budget_close=False):
        self.server, self.w = server, w
        self.caps = caps(w)
        self.dims = [P.dims(n) for n in w.n_items]
        self.sessions = [server.open(X, Y, w.ks[g], self.caps[g])
                         for g, (X, Y) in enumerate(self.dims)]
        self.bufs = [w.request_reads(i) for i in range(len(w.requests))]
        self.outs = {}
        self.last = {}
        for i, q in enumerate(w.requests):
            self.last[q.genome] = i
        self.budget_close = budget_close

    def submit(self, i):
        q = self.w.requests[i]
        reads, offs = self.bufs[i]
        kw = {}
        if q.classify:
            cap = self.caps[q.genome]
            self.outs[i] = (torch.empty(cap, dtype=torch.int64, device="cuda"),
                            torch.empty(cap, dtype=torch.int64, device="cuda"))
            kw = {"classify": True, "tau": q.tau, "trust": self.outs[i][0],
                  "err": self.outs[i][1]}
        return self.server.submit(self.sessions[q.genome], reads, offs, **kw)

    def outputs(self, i, r):
        """The request's outputs as host arrays (reads its session's list)."""
        q = self.w.requests[i]
        assert r["status"] == 0, f"request {i}: status {r['status']}"
        o = {"nw": r["n_windows"], "first": r["distinct_first"],
             "new": self.server.read_distinct(self.sessions[q.genome], r["distinct_first"],
                                              r["n_new"])}
        if q.classify:
            t, e = self.outs[i]
            o["trust"] = t[:r["n_trust"]].cpu().numpy().view(np.uint64).copy()
            o["err"] = e[:r["n_err"]].cpu().numpy().view(np.uint64).copy()
        return o


def run_mix(w, **cfg):
    lane_bases = max(w.request_bases(i) for i in range(len(w.requests)))
    lane_reads = max(q.n_reads for q in w.requests)
    server = P.Server(memory_budget=cfg.pop("budget", 1 << 34), lane_bases=lane_bases,
                      lane_reads=lane_reads, **cfg)
    return server


def test_alone_equals_mix_equals_oracle(workload):
    w = workload
    print(f"case serving mix: {len(w.requests)} requests, 16 sessions", flush=True)
    mix = run_mix(w, lane_requests=16, lanes=2)
    cm = Client(mix, w)
    # arrivals 100x denser than the trace's, so that requests arrive while
    # others run and share batches
    res_mix = serve.replay(mix, [q.t * 0.01 for q in w.requests], cm.submit)
    out_mix = [cm.outputs(i, r) for i, r in enumerate(res_mix)]
    st = mix.stats()
    assert st["requests_done"] == len(w.requests)
    assert st["batched_requests"] > 0 and st["max_batch"] >= 2, st
    assert st["plain_requests"] == 0 and st["lanes_in_flight_max"] == 2, st
    words_mix = [mix.read_words(s, X * Y) for s, (X, Y) in zip(cm.sessions, cm.dims)]

    print("case serving alone: one request per batch, in order", flush=True)
    alone = run_mix(w, lane_requests=1, lanes=1)
    ca = Client(alone, w)
    out_alone = []
    for i in range(len(w.requests)):
        tk = ca.submit(i)
        alone.wait(tk)
        out_alone.append(ca.outputs(i, alone.result(tk)))
    st_alone = alone.stats()
    assert st_alone["max_batch"] == 1 and st_alone["lanes_in_flight_max"] == 1, st_alone
    for i, (a, m) in enumerate(zip(out_alone, out_mix)):
        assert a["nw"] == m["nw"] and a["first"] == m["first"], f"request {i}"
        assert np.array_equal(a["new"], m["new"]), f"request {i}: new distinct"
        if "trust" in a:
            assert np.array_equal(a["trust"], m["trust"]), f"request {i}: trust"
            assert np.array_equal(a["err"], m["err"]), f"request {i}: err"

    print("case serving oracle, session by session", flush=True)
    bfs = [oracle.CountBF(X, Y) for X, Y in cm.dims]
    dist = [np.zeros(0, dtype=np.uint64) for _ in bfs]
    for i, q in enumerate(w.requests):
        reads, offs = cm.bufs[i]
        d, nw = bfs[q.genome].insert(reads, offs, w.ks[q.genome])
        m = out_mix[i]
        assert m["nw"] == nw, f"request {i}: windows"
        assert m["first"] == len(dist[q.genome]), f"request {i}: first"
        assert np.array_equal(m["new"], d), f"request {i}: distinct"
        dist[q.genome] = np.concatenate([dist[q.genome], d])
        if q.classify:
            t, e = bfs[q.genome].classify(dist[q.genome], q.tau)
            assert np.array_equal(m["trust"], t), f"request {i}: trust"
            assert np.array_equal(m["err"], e), f"request {i}: err"
    for g, bf in enumerate(bfs):
        assert np.array_equal(words_mix[g], bf.words), f"session {g}: words"
    mix.close_server()
    alone.close_server()


def test_admission_by_memory(workload):
    """A budget of about three sessions: later sessions wait, are admitted as
    earlier ones close after their last request, and still give the oracle's
    outputs."""
    w = workload
    dims = [P.dims(n) for n in w.n_items]
    need = sorted(X * Y * 8 + 8 * c + 8 for (X, Y), c in zip(dims, caps(w)))
    budget = sum(need[-3:])
    server = run_mix(w, budget=budget, lane_requests=8, lanes=2)
    c = Client(server, w)
    st0 = server.stats()
    assert st0["sessions_waiting"] > 0 and st0["session_bytes"] <= budget
    seen_waiting = [st0["sessions_waiting"]]
    closed = set()

    def after(i, tk):
        g = w.requests[i].genome
        if c.last[g] == i:
            server.close(c.sessions[g])
            closed.add(g)
        s = server.stats()
        assert s["session_bytes"] <= budget
        seen_waiting.append(s["sessions_waiting"])

    # sessions without requests close at once
    for g in range(len(dims)):
        if g not in c.last:
            server.close(c.sessions[g])
    print("case serving admission: budget", budget, flush=True)
    # arrivals compressed so that requests queue behind waiting sessions
    res = serve.replay(server, [q.t * 0.2 for q in w.requests], c.submit, on_submitted=after)
    assert all(r is not None and r["done"] for r in res)
    # outputs after close cannot be read back from the server: compare the
    # counts with an oracle run
    bfs = [oracle.CountBF(X, Y) for X, Y in dims]
    dist = [np.zeros(0, dtype=np.uint64) for _ in bfs]
    for i, q in enumerate(w.requests):
        reads, offs = c.bufs[i]
        d, nw = bfs[q.genome].insert(reads, offs, w.ks[q.genome])
        assert res[i]["status"] == 0
        assert res[i]["n_windows"] == nw and res[i]["n_new"] == len(d), f"request {i}"
        assert res[i]["distinct_first"] == len(dist[q.genome])
        dist[q.genome] = np.concatenate([dist[q.genome], d])
        if q.classify:
            t, e = bfs[q.genome].classify(dist[q.genome], q.tau)
            assert res[i]["n_trust"] == len(t) and res[i]["n_err"] == len(e), f"request {i}"
    st = server.stats()
    assert st["sessions_open"] == 0 and st["session_bytes"] == 0
    assert max(seen_waiting) > 0
    server.close_server()


def test_request_errors(workload):
    w = workload
    server = P.Server(memory_budget=1 << 30, lane_bases=1 << 20, lane_reads=1 << 14,
                      lane_requests=4, lanes=2)
    X, Y = P.dims(20_000)
    s = server.open(X, Y, 21, 64)  # room for 64 distinct k-mers only
    reads, offs = w.request_reads(0)
    reads, offs = np.ascontiguousarray(reads[:int(offs[40])]), offs[:41].copy()
    tk = server.submit(s, reads, offs)
    server.wait(tk)
    r = server.result(tk)
    assert r["done"] and r["status"] == P.kmerco.KC_ERANGE and r["n_new"] > 64
    server.release(tk)
    with pytest.raises(P.KmercoError):
        server.result(tk)  # released
    with pytest.raises(P.KmercoError):
        server.release(tk)
    bad = offs.copy()
    bad[5], bad[6] = bad[6], bad[5]
    with pytest.raises(P.KmercoError):
        server.submit(s, reads, bad)  # offsets not monotone
    bad = offs + np.uint64(1)
    with pytest.raises(P.KmercoError):
        server.submit(s, reads, bad)  # offsets[0] != 0
    big = np.zeros(2, dtype=np.uint64)
    big[1] = (1 << 20) + 1
    with pytest.raises(P.KmercoError):
        server.submit(s, np.zeros(big[1], dtype=np.uint8), big)  # beyond the lane
    with pytest.raises(P.KmercoError):
        server.open(*P.dims(5e9), 31, 10)  # more than the whole budget
    server.close(s)
    with pytest.raises(P.KmercoError):
        server.submit(s, reads, offs)  # closed session
    server.close_server()


def test_full_scale_trace_against_oracle_digests():
    """The whole serving trace at full size (247 requests, 16.1 Gbases, 16
    sessions of 75-505 MB), all requests submitted at once on two lanes:
    every request's inserted and first-seen counts and classification
    counts, every session's final countBF words and distinct list, and each
    session's last classification equal the oracle's (digests written by
    tests/golden/make_digests.py serving)."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "serving_digests.json")
    if not os.path.exists(path):
        pytest.skip("no oracle digests for the serving trace")
    ref = json.load(open(path))

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()

    print("case serving full scale: generating the trace", flush=True)
    w = synth.serving_workload(duration_s=ref["duration_s"])
    assert len(w.requests) == ref["n_requests"]
    dims = [P.dims(n) for n in w.n_items]
    cap = [int(math.ceil(1.2 * d)) + 4096 for d in w.expected_distinct]
    server = P.Server(memory_budget=200 * 10**9,
                      lane_bases=max(w.request_bases(i) for i in range(len(w.requests))),
                      lane_reads=max(q.n_reads for q in w.requests), lane_requests=64, lanes=2)
    sessions = [server.open(X, Y, w.ks[g], cap[g]) for g, (X, Y) in enumerate(dims)]
    outs = [(torch.empty(c, dtype=torch.int64, device="cuda"),
             torch.empty(c, dtype=torch.int64, device="cuda")) for c in cap]
    bufs = [w.request_reads(i) for i in range(len(w.requests))]

    def submit(i):
        q = w.requests[i]
        kw = {}
        if q.classify:
            kw = {"classify": True, "tau": q.tau, "trust": outs[q.genome][0],
                  "err": outs[q.genome][1]}
        return server.submit(sessions[q.genome], bufs[i][0], bufs[i][1], **kw)

    print("case serving full scale: all requests at once", flush=True)
    res = serve.replay(server, [0.0] * len(w.requests), submit)
    for s in ref["sessions"]:
        g = s["session"]
        X, Y = dims[g]
        assert (s["X"], s["Y"], s["k"]) == (X, Y, w.ks[g]), f"session {g}: layout"
        for r in s["requests"]:
            got = res[r["request"]]
            assert got["status"] == 0, f"request {r['request']}: status"
            assert (got["n_windows"], got["n_new"]) == (r["n_windows"], r["n_new"]), \
                f"request {r['request']}: counts"
            if "n_trust" in r:
                assert (got["n_trust"], got["n_err"]) == (r["n_trust"], r["n_err"]), \
                    f"request {r['request']}: classification counts"
        assert sha(server.read_words(sessions[g], X * Y)) == s["words_sha256"], f"session {g}"
        assert sha(server.read_distinct(sessions[g], 0, s["n_distinct"])) == \
            s["distinct_sha256"], f"session {g}: distinct list"
        lc = s["last_classify"]
        if lc:
            nt, ne = res[lc["request"]]["n_trust"], res[lc["request"]]["n_err"]
            t, e = outs[g]
            assert sha(t[:nt].cpu().numpy().view(np.uint64)) == lc["trust_sha256"], f"session {g}"
            assert sha(e[:ne].cpu().numpy().view(np.uint64)) == lc["err_sha256"], f"session {g}"
    server.close_server()
