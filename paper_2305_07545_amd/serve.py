"""Client side of the serving form: replay timed requests against a Server.

The loop submits each request at its arrival time (on the server's clock),
pumps the server (which retires, admits and issues batches natively) and
collects every request's result when it is done.  Latency of a request is
t_done - t_submit on the server's clock.
"""
from __future__ import annotations

import time


def replay(server, arrivals, submit, on_submitted=None, idle_sleep_s: float = 50e-6,
           stall_s: float = 120.0):
    """arrivals: ascending arrival times (s from start); submit(i) submits
    request i and returns its ticket; on_submitted(i, ticket) is called after
    each submit (e.g. to close a session after its last request).  Returns the
    results in request order.  Raises if no request completes for stall_s
    seconds while some are pending."""
    n = len(arrivals)
    tickets = [0] * n
    results = [None] * n
    pending = []
    t0 = server.now()
    last_progress = t0
    i = 0
    while i < n or pending:
        if pending and server.now() - last_progress > stall_s:
            raise RuntimeError(f"serving stalled: {len(pending)} requests pending")
        now = server.now() - t0
        while i < n and arrivals[i] <= now:
            if not pending:
                last_progress = server.now()
            tickets[i] = submit(i)
            pending.append(i)
            if on_submitted is not None:
                on_submitted(i, tickets[i])
            i += 1
        if server.pump() or pending:
            still = []
            for j in pending:
                r = server.result(tickets[j])
                if r["done"]:
                    results[j] = r
                    server.release(tickets[j])
                else:
                    still.append(j)
            progressed = len(still) < len(pending)
            pending = still
            if progressed:
                last_progress = server.now()
                continue
        if i < n and not pending:
            # idle until the next arrival
            wait = arrivals[i] - (server.now() - t0)
            if wait > 0:
                time.sleep(min(wait, 1e-3))
        else:
            time.sleep(idle_sleep_s)
    return results


def latency_summary(results) -> dict:
    """p50 / p99 / mean / max latency (ms) over done results."""
    import numpy as np
    lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in results if r is not None])
    if len(lat) == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "n": int(len(lat))}
