"""Poisson-trace driver for the continuous-batching server.

Replays a request trace (arrival times, ensembles, t_end, dt) against
fewbody.Server in real time: each request is submitted at its arrival time
on the monotonic clock, and its latency is completion minus arrival.
Reports p50/p99 latency (nearest rank), offered and achieved load, and the
aggregate system-steps/s over the makespan.
"""
from __future__ import annotations

import math
import time

import numpy as np


def nearest_rank(values, q):
    """q-th percentile by the nearest-rank method (q in (0, 100])."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * v.size)))
    return float(v[k - 1])


def request_steps(t_end, dt):
    """Steps the server takes for one request from t = 0 (whole steps, plus a
    shortened last one unless the remainder is below 1e-9 dt)."""
    span = t_end / dt
    nf = int(math.floor(span)) if span > 0 else 0
    while nf > 0 and (nf * dt - t_end) * dt > 0:
        nf -= 1
    rem = t_end - nf * dt
    return nf + (1 if rem * dt > 1e-9 * dt * dt else 0)


def run_trace(fb, trace, budget_bytes=0, max_resident=0, steps_per_quantum=0, keep_results=False,
              log=None, policy=0, quantum_tiles=0, chunk_slots=0, long_steps=0, idle_spread=0):
    """Replay `trace` (list of gen.Request) in real time; returns a report dict."""
    srv = fb.Server(budget_bytes, max_resident, steps_per_quantum, policy=policy,
                    quantum_tiles=quantum_tiles, chunk_slots=chunk_slots, long_steps=long_steps,
                    idle_spread=idle_spread)
    try:
        t0 = fb.monotonic()
        ids = []
        for r in trace:
            delay = t0 + r.arrival - fb.monotonic()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit_gen(r.ensemble, r.t_end, r.dt))
        lat, queue_wait, results = [], [], []
        steps_total = 0.0
        last_done = t0
        for k, (rid, r) in enumerate(zip(ids, trace)):
            st = srv.wait(rid)
            if st != fb.REQ_DONE:
                raise RuntimeError(f"request {rid} ended in state {st}")
            res = srv.result(rid)
            arrival = t0 + r.arrival
            lat.append(res["t_done"] - arrival)
            queue_wait.append(res["t_admit"] - arrival)
            last_done = max(last_done, res["t_done"])
            steps_total += r.ensemble.n_sys * request_steps(r.t_end, r.dt)
            if keep_results:
                results.append(res)
            if log and (k + 1) % max(1, len(trace) // 10) == 0:
                log(f"[serve] {k + 1}/{len(trace)} requests done")
        stats = srv.stats()
    finally:
        srv.close()
    makespan = last_done - t0
    span_arrivals = trace[-1].arrival - trace[0].arrival if len(trace) > 1 else 0.0
    offered = steps_total / span_arrivals if span_arrivals > 0 else float("nan")
    out = {
        "requests": len(trace),
        "p50_latency_s": nearest_rank(lat, 50),
        "p99_latency_s": nearest_rank(lat, 99),
        "max_latency_s": float(np.max(lat)) if lat else float("nan"),
        "p50_queue_wait_s": nearest_rank(queue_wait, 50),
        "makespan_s": makespan,
        "system_steps": steps_total,
        "aggregate_system_steps_per_s": steps_total / makespan if makespan > 0 else float("nan"),
        "offered_system_steps_per_s": offered,
        "quanta": stats["quanta"],
        "spread_quanta": stats["spread_quanta"],
        "busy_fraction": stats["busy_seconds"] / makespan if makespan > 0 else float("nan"),
        "peak_device_bytes": stats["peak_bytes"],
    }
    if keep_results:
        out["results"] = results
        out["latencies"] = lat
    return out
