"""Serving driver: replay a stream of reconstruction requests through the
native server (spect_server_*, continuous batching) or one at a time through
plain osem_reconstruct calls, and record per-request latency.

A trace is a list of (arrival time in seconds, request class); a request
class bundles a plan, its data sets and the OSEM schedule.  The driver
submits each request when the wall clock reaches its arrival time (the f of
a request is a fresh image of ones), polls the server between arrivals, and
records completion at the first poll that sees the request done.  Latency =
completion - arrival.  The one-at-a-time baseline runs each request when it
has arrived and the previous one has finished.
"""
from __future__ import annotations

import sys
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from ._binding import REQ_DONE, REQ_FAILED, Plan, Server, SpectError


@dataclass
class RequestClass:
    name: str
    plan: Plan
    data: List[torch.Tensor]                 # measured projections to cycle through
    mu: Optional[List[torch.Tensor]] = None  # attenuation maps, one per data set
    n_iters: int = 4
    n_subsets: int = 8


@dataclass
class Served:
    cls: int
    arrival: float
    submitted: float
    done: float = float("nan")
    f: Optional[torch.Tensor] = None
    data_index: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_trace(rate_per_s: float, duration_s: float, n_classes: int, rng: np.random.Generator,
                  weights: Optional[Sequence[float]] = None) -> List[Tuple[float, int]]:
    """Arrival times of a Poisson process with the given rate over duration_s
    seconds, each with a class drawn with the given weights (uniform by default)."""
    out, t = [], 0.0
    p = None if weights is None else np.asarray(weights, float) / np.sum(weights)
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return out
        out.append((t, int(rng.choice(n_classes, p=p))))


class _Progress:
    """A line on stderr every `every_s` seconds of a long replay (0: never)."""

    def __init__(self, every_s: float, what: str, total: int):
        self.every, self.what, self.total = every_s, what, total
        self.next = every_s

    def __call__(self, now: float, done: int):
        if self.every > 0 and now >= self.next:
            print(f"{self.what}: {done}/{self.total} requests done after {now:.0f} s", file=sys.stderr, flush=True)
            self.next += self.every


def replay(server: Server, classes: Sequence[RequestClass], trace: Sequence[Tuple[float, int]],
           keep_images: bool = False, poll_sleep_s: float = 2e-4, log_every_s: float = 0.0) -> List[Served]:
    """Run the trace in real time; returns one record per request."""
    served: List[Served] = []
    pending = {}
    counters = [0] * len(classes)
    progress = _Progress(log_every_s, "server replay", len(trace))
    t0 = time.perf_counter()
    i = 0
    while i < len(trace) or pending:
        progress(time.perf_counter() - t0, len(served) - len(pending))
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i][0] <= now:
            arrival, c = trace[i]
            rc = classes[c]
            k = counters[c] % len(rc.data)
            counters[c] += 1
            f = torch.ones(rc.plan.object_shape, dtype=torch.float32, device="cuda")
            rid = server.submit(rc.plan, f, rc.data[k], rc.n_iters, rc.n_subsets,
                                None if rc.mu is None else rc.mu[k])
            rec = Served(c, arrival, time.perf_counter() - t0, f=f, data_index=k)
            served.append(rec)
            pending[rid] = rec
            i += 1
        server.progress()
        now = time.perf_counter() - t0
        for rid in list(pending):
            st = server.status(rid)
            if st == REQ_DONE:
                rec = pending.pop(rid)
                rec.done = now
                server.forget(rid)
                if not keep_images:
                    rec.f = None
            elif st == REQ_FAILED:  # status raises for failed requests; kept for clarity
                raise SpectError(-3, f"request {rid} failed")
        if pending or i < len(trace):
            nxt = trace[i][0] if i < len(trace) else None
            if nxt is None or nxt - (time.perf_counter() - t0) > poll_sleep_s:
                time.sleep(poll_sleep_s)
    return served


def replay_one_at_a_time(classes: Sequence[RequestClass], trace: Sequence[Tuple[float, int]],
                         keep_images: bool = False, log_every_s: float = 0.0) -> List[Served]:
    """The baseline: each request is one osem_reconstruct call on the current
    stream, started when it has arrived and the previous one has finished."""
    served: List[Served] = []
    counters = [0] * len(classes)
    progress = _Progress(log_every_s, "one-at-a-time replay", len(trace))
    t0 = time.perf_counter()
    for arrival, c in trace:
        progress(time.perf_counter() - t0, len(served))
        wait = arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        rc = classes[c]
        k = counters[c] % len(rc.data)
        counters[c] += 1
        f = torch.ones(rc.plan.object_shape, dtype=torch.float32, device="cuda")
        rec = Served(c, arrival, time.perf_counter() - t0, f=f, data_index=k)
        rc.plan.reconstruct(rc.data[k], rc.n_iters, rc.n_subsets, None if rc.mu is None else rc.mu[k], f=f)
        torch.cuda.synchronize()
        rec.done = time.perf_counter() - t0
        if not keep_images:
            rec.f = None
        served.append(rec)
    return served


def summary(served: Sequence[Served], wall_s: Optional[float] = None) -> dict:
    lat = np.array([s.latency for s in served]) * 1e3
    end = max(s.done for s in served) if served else 0.0
    wall = wall_s if wall_s is not None else end
    return {"requests": len(served), "recon_per_s": len(served) / wall if wall > 0 else float("nan"),
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_mean": float(lat.mean()), "latency_ms_max": float(lat.max())}
