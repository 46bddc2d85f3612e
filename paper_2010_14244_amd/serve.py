"""Continuous-batching serving loop over gmacop_server_step.

Queries arrive on a seeded Poisson clock; at every step the loop admits
the queries that have arrived into free slots (as many as fit), advances
every in-flight query by one iteration on the GPU, and records the
completion time of the queries that finished.  Latency = completion -
arrival, so it includes queueing for a free slot.
"""
from __future__ import annotations

import time

import numpy as np

from . import gmacop


def poisson_arrivals(n: int, rate_qps: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds from start) of n queries at the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate_qps, size=n))


def serve(server: "gmacop.Server", od: np.ndarray, arrivals: np.ndarray, *, warmup: int = 0,
          stream=None, log=None) -> dict:
    """Serve queries od[i] = (qid, src, dst) arriving at arrivals[i] (sorted).
    Returns per-query latency (s), p50/p99 over the queries after the first
    `warmup` ones, and the sustained completion rate over the measured part.

    Admission is first come, first served, so the queries waiting for a slot
    are always the index range [head, nxt): each step hands the server only
    as many of them as it has free slots, and the host work of a step does
    not grow with the backlog."""
    n = od.shape[0]
    od = np.ascontiguousarray(od, np.uint32)
    done_at = np.full(n, np.nan)
    results = {}
    qid_to_idx = {int(od[i, 0]): i for i in range(n)}
    steps = 0
    head = nxt = 0           # arrived and waiting: [head, nxt)
    in_flight = 0
    t0 = time.perf_counter()
    completed = 0
    while completed < n:
        now = time.perf_counter() - t0
        nxt = max(nxt, int(np.searchsorted(arrivals, now, side="right")))
        if head == nxt and in_flight == 0:
            # idle: wait for the next arrival
            if nxt < n:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
            continue
        k = max(0, min(nxt - head, server.slots - in_flight))
        admitted, done = server.step(od[head:head + k], stream)
        head += admitted
        in_flight += admitted - len(done)
        t_done = time.perf_counter() - t0
        for qid, path, cost in done:
            i = qid_to_idx[qid]
            done_at[i] = t_done
            results[qid] = (path, cost)
        completed += len(done)
        steps += 1
        if log and steps % 50 == 0:
            log(f"[serve] step {steps}: t={t_done:.2f}s done={completed}/{n} in_flight={in_flight} "
                f"queued={nxt - head}")
    lat = done_at - arrivals
    meas = slice(warmup, n)
    span = np.nanmax(done_at[meas]) - arrivals[warmup] if n > warmup else float("nan")
    arr_span = float(arrivals[-1] - arrivals[0]) if n > 1 else 0.0
    return dict(latency_s=lat, results=results, steps=steps,
                p50_ms=float(np.percentile(lat[meas], 50) * 1e3), p99_ms=float(np.percentile(lat[meas], 99) * 1e3),
                sustained_qps=float((n - warmup) / span),
                offered_qps=(n - 1) / arr_span if arr_span > 0 else float("inf"),
                wall_s=float(time.perf_counter() - t0))
