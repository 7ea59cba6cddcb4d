"""Serving driver: replay a seeded Poisson arrival stream against hs_server.

Requests are layered random circuits (U3 on every qubit + a CX matching per
layer) with n ~ U{lo..hi} and depth ~ U{lo..hi} layers, complex64 with
probability 0.7, else complex128.  Each request is submitted at its arrival
time with that time as its arrival stamp on the server clock, so a request's
latency runs from its scheduled arrival to its observed completion and
includes the host work (partition, compile, descriptor upload) and any
queueing.  The native server prepares requests on its own host threads,
admits them by state bytes against the budget and runs them concurrently
with whatever is resident.
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


def run_stream(requests, budget_bytes: int = 0, num_streams: int = 4, read_states: bool = False,
               time_scale: float = 1.0, strategy: str = "closure"):
    """Submit `requests` (workloads.Request) at their arrival times.

    Returns a dict: per-request latency (s) and its four parts (host queue,
    preparation, admission wait, device), total wall time, server stats,
    and, with read_states, every request's full final state.
    """
    circuits = [wl.layered28(r.seed, n=r.n, layers=r.layers) for r in requests]
    srv = hisv.Server(budget_bytes, num_streams)
    tickets = []
    t0 = srv.clock()
    for r, (n, gates) in zip(requests, circuits):
        target = t0 + r.arrival_s * time_scale
        while True:
            now = srv.clock()
            if now >= target:
                break
            time.sleep(min(0.001, target - now))
        tickets.append(srv.submit(n, gates, r.dtype, 0, part_limit(n, r.dtype), strategy,
                                  arrival_s=target))
    lat, parts, states = [], [], []
    for t, r in zip(tickets, requests):
        srv.wait(t)
        lat.append(srv.latency(t))
        parts.append(srv.timing(t))
        if read_states:
            states.append(srv.amplitudes(t, 0, 1 << r.n))
        srv.release(t)
    wall = srv.clock() - t0
    stats = srv.stats()
    srv.close()
    return {"latency": np.array(lat), "parts": np.array(parts), "wall": wall, "stats": stats,
            "states": states}


def summarize(res: dict, n_req: int) -> dict:
    """p50 / p99 latency, circuits/s, and where the p50 and p99 requests'
    time went (host = queue + preparation; admission wait; device)."""
    lat, parts = res["latency"], res["parts"]
    out = {
        "requests": int(n_req),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(np.mean(lat) * 1e3),
        "circuits_per_s": float(n_req / res["wall"]),
    }
    order = np.argsort(lat)
    for name, q in (("p50", 50), ("p99", 99)):
        i = order[min(len(lat) - 1, int(round(q / 100 * (len(lat) - 1))))]
        host_queue, prep, admit, dev = parts[i]
        out[f"{name}_request_ms"] = {"host_queue": host_queue * 1e3, "prepare": prep * 1e3,
                                     "admission_wait": admit * 1e3, "device": dev * 1e3}
    tot = parts.sum(axis=0)
    out["host_share"] = float((tot[0] + tot[1]) / max(tot.sum(), 1e-30))
    out["prepare_ms_mean"] = float(np.mean(parts[:, 1]) * 1e3)
    return out
