"""Serving loop over a pool: continuous batching of square-lattice solves.

Requests (grid side, step count, Riemann states) arrive over wall-clock time.
The loop admits every arrived request that fits (a free slot and room for its
footprint in the pool's arena; first come, first served, so a large request at
the head waits for memory rather than being overtaken), advances all admitted
solves together by `tick` pool steps (one persistent launch per step, HIP-graph
captured), then collects the finished ones, whose slots and memory go to the
next arrivals.  Work of different requests overlaps inside each launch.

The device never waits for the host: each tick is queued with a progress
snapshot behind it, and the host reads the previous tick's snapshot (finished
slots, their totals) while the next tick runs.  Admissions and releases are
stream-ordered, so they take effect from the next tick queued.

Latency of a request = completion (its result collected) - arrival.
Aggregate throughput = sum over requests of nodes x steps / makespan.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs
from .lbsd import LB_POOL_FREE, Pool


def request_footprint(pool: Pool, side: int) -> int:
    return pool.footprint(side, side)


def run(pool: Pool, requests, *, tick: int = 25, fetch: str = "totals", time_scale: float = 1.0,
        on_result=None):
    """Serve `requests` (dicts from inputs.serve_requests) on `pool`.

    fetch: "totals" (conservation totals), "moments" (host copy of the
    fields) or "none".  on_result(i, result) is called per finished request.
    Returns a dict of per-request latencies and aggregate figures."""
    n = len(requests)
    for r in requests:
        if request_footprint(pool, r["side"]) > pool.arena_bytes:
            raise ValueError(f"request of side {r['side']} can never fit the arena")
    arrival = np.array([r["arrival"] for r in requests]) * time_scale
    admitted = np.full(n, np.nan)
    finished = np.full(n, np.nan)
    live = {}  # slot -> request index
    nxt = 0
    t0 = time.perf_counter()
    ticks = 0
    pending = []  # snapshots queued and not read yet (sequence numbers; buffer = seq % 2)
    seq = 0
    while nxt < n or live or pending:
        now = time.perf_counter() - t0
        if not live and not pending and nxt < n and arrival[nxt] > now:
            time.sleep(arrival[nxt] - now)  # idle until the next arrival
            now = time.perf_counter() - t0
        while nxt < n and arrival[nxt] <= now:
            r = requests[nxt]
            slot = pool.admit_riemann(r["side"], r["x_d"], r["left"], r["right"], r["steps"], ny=r["side"],
                                      lam=inputs.cfl_lambda([r["left"], r["right"]]))
            if slot is None:
                break  # no room yet: the head of the queue waits
            live[slot] = nxt
            admitted[nxt] = time.perf_counter() - t0
            nxt += 1
        queued = False
        if live and len(pending) < 2:
            pool.advance(tick)
            pool.snapshot(seq % 2)
            pending.append(seq)
            seq += 1
            ticks += 1
            queued = True
        if not pending:
            continue
        if queued and len(pending) < 2:
            continue  # keep one tick queued ahead before waiting for a snapshot
        s = pending.pop(0)
        done, status, tot = pool.snapshot_read(s % 2)
        for slot in [q for q in live if status[q] not in (0, LB_POOL_FREE)]:
            i = live.pop(slot)
            if status[slot] != 1:
                raise RuntimeError(f"request {i} failed with status {status[slot]} after {done[slot]} steps")
            if fetch == "totals":
                res = tot[slot].copy()
            elif fetch == "moments":
                res = pool.moments(slot)
            else:
                res = None
            finished[i] = time.perf_counter() - t0
            pool.release(slot)
            if on_result is not None:
                on_result(i, res)
    makespan = time.perf_counter() - t0
    lat = finished - arrival
    work = float(sum(r["side"] ** 2 * r["steps"] for r in requests))
    return dict(latency_s=lat, queue_s=admitted - arrival, makespan_s=makespan, ticks=ticks,
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                node_updates=work, nups=work / makespan)


def fill(pool: Pool, requests, steps: int):
    """Admit requests in order until the pool is full; returns (slots, nodes)."""
    slots, nodes = [], 0
    for r in requests:
        s = pool.admit_riemann(r["side"], r["x_d"], r["left"], r["right"], steps, ny=r["side"],
                               lam=inputs.cfl_lambda([r["left"], r["right"]]))
        if s is None:
            break
        slots.append(s)
        nodes += r["side"] ** 2
    return slots, nodes


def calibrate(pool: Pool, requests, steps: int = 30, trials: int = 3, windows: int = 3, warm: int = 150):
    """Fill the pool with the first requests that fit, pick the tile shape
    with the pool's autotuner, run `warm` steps (the first steps after a
    Riemann start run up to 1.6x slower than the developed flow a request
    spends most of its 100-5000 steps in), and measure node-updates/s over
    `windows` windows of `steps` steps (the median window).  Returns
    (node-updates/s, chosen shape); the pool is left empty."""
    slots, nodes = fill(pool, requests, 2 + warm + (windows + 1) * steps)
    pool.advance(2)
    shape, _ = pool.autotune(trials=trials)
    pool.advance(warm)
    ms = sorted(pool.advance_timed(steps) for _ in range(windows))[windows // 2]
    for s in slots:
        pool.release(s)
    return nodes * steps / (ms * 1e-3), shape
