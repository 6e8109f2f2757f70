"""Session driver for the request scheduler (hmv_server_*).

A Lanczos iteration issues matvecs with one fixed matrix, each after the
previous one finished; a session here is such a closed loop of matvecs.
Sessions arrive over time (Poisson), are bound to one resident matrix, and
submit their next matvec as soon as the previous one is retired.  The
scheduler (C++) admits requests as stream slots and pool memory free up, so
requests from many sessions overlap on the device.

This module only drives the scheduler and records timings; all arithmetic
runs in the library.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field


@dataclass
class Session:
    sid: int
    matrix_id: int
    arrival: float                    # seconds after the start
    xs: list                          # device tensors, one per matvec
    ys: list                          # device tensors, one per matvec (may repeat)
    next_k: int = 0
    inflight: int = -1                # request id in flight, -1 if none
    submit_t: float = 0.0
    latencies: list = field(default_factory=list)
    done_at: float = -1.0


def poisson_arrivals(rate: float, count: int, rng) -> list:
    """count arrival times of a Poisson process of the given rate (per s)."""
    t, out = 0.0, []
    for _ in range(count):
        t += -math.log(1.0 - rng.random()) / rate
        out.append(t)
    return out


def run(server, sessions: list, poll_sleep: float = 2e-5, on_done=None, time_limit: float = 600.0):
    """Drive all sessions to completion.  Returns (wall seconds, latencies,
    per-request (session, k, latency, status) records).  on_done(session, k)
    is called when request k of a session is retired."""
    pending = sorted(sessions, key=lambda s: s.arrival)
    by_rid = {}
    active = []
    records = []
    t0 = time.perf_counter()
    while pending or active:
        now = time.perf_counter() - t0
        if now > time_limit:
            raise RuntimeError("serving run exceeded its time limit")
        while pending and pending[0].arrival <= now:
            s = pending.pop(0)
            active.append(s)
        for s in active:
            if s.inflight < 0 and s.next_k < len(s.xs):
                s.submit_t = time.perf_counter()
                rid = server.submit(s.matrix_id, s.sid, s.xs[s.next_k], s.ys[s.next_k])
                s.inflight = rid
                by_rid[rid] = s
        for rid, status in server.poll():
            t = time.perf_counter()
            s = by_rid.pop(rid)
            lat = t - s.submit_t
            s.latencies.append(lat)
            records.append((s.sid, s.next_k, lat, status))
            if on_done is not None:
                on_done(s, s.next_k)
            s.next_k += 1
            s.inflight = -1
            if s.next_k >= len(s.xs):
                s.done_at = t - t0
        active = [s for s in active if s.done_at < 0]
        if poll_sleep:
            time.sleep(poll_sleep)
    wall = time.perf_counter() - t0
    lats = [r[2] for r in records]
    return wall, lats, records


def percentile(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))
    return v[k]
