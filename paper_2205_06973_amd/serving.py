"""Serving driver: replay a seeded Poisson arrival stream against hs_server.

Requests are layered random circuits (U3 on every qubit + a CX matching per
layer) with n ~ U{lo..hi} and depth ~ U{lo..hi} layers, complex64 with
probability 0.7, else complex128.  Each request is submitted at its arrival
time; the native server admits it by state bytes against the budget, runs it
concurrently with whatever is resident, and the driver collects per-request
latency (submit to completion) for p50/p99 and circuits/s.
"""

from __future__ import annotations

import time

import numpy as np

from . import hisv
from . import workloads as wl


def part_limit(n: int, dtype: str) -> int:
    """Whole state in one tile when it fits, else the widest part the kernel takes."""
    whole = 14 if dtype == "c64" else 13
    return n if n <= whole else hisv.hs_max_part_qubits(dtype)


def run_stream(requests, budget_bytes: int = 0, num_streams: int = 4, read_check: int = 0,
               time_scale: float = 1.0, strategy: str = "greedy"):
    """Submit `requests` (workloads.Request) at their arrival times.

    Returns per-request latencies (s), total wall time, server stats and the
    first `read_check` amplitudes of every request (for mixed-vs-alone checks).
    """
    srv = hisv.Server(budget_bytes, num_streams)
    tickets = []
    t0 = time.perf_counter()
    for r in requests:
        target = t0 + r.arrival_s * time_scale
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(0.001, target - now))
        n, gates = wl.layered28(r.seed, n=r.n, layers=r.layers)
        tickets.append(srv.submit(n, gates, r.dtype, 0, part_limit(n, r.dtype), strategy))
    lat, amps = [], []
    for t in tickets:
        srv.wait(t)
        lat.append(srv.latency(t))
        if read_check:
            amps.append(srv.amplitudes(t, 0, read_check))
        srv.release(t)
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    return np.array(lat), wall, stats, amps


def summarize(lat: np.ndarray, wall: float, n_req: int) -> dict:
    return {
        "requests": int(n_req),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "circuits_per_s": float(n_req / wall),
    }
