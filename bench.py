#!/usr/bin/env python3
"""Benchmark of the partitioned state-vector hot path on one MI355X.

A step is one pass of the whole path over one circuit: the gate list is
loaded, partitioned (closure partitioner: each part's qubit set chosen so
that the gates it can take from the current front weigh most; --strategy
picks Nat, DFS or dagP of Sec. IV.B, or the greedy ready-set partitioner,
instead) and compiled (the specialized part
kernels come from the kernel cache after the first pass), every part is
applied as one in-place Gather-Execute-Scatter sweep of a state resident in
HBM (Alg. 1), and the FP64 norm is read back.  Default workload: a 33-qubit
random circuit of 1,000 gates drawn uniformly from {H, RZ, RX, CX, CZ},
complex128 state (the paper's 16 bytes per amplitude, Sec. II.B; 128 GiB),
acyclic partition with at most k = 7 qubits per part.

Prints ONE JSON line on stdout:
  value      gates/s over the timed steps (wall clock, synchronized; host
             ingest, partition and compile included)
  roofline   the part-pass kernel: algorithmic bytes per launch (read + write
             every amplitude once: 2 * 2^n * bytes/amplitude) / the average
             launch duration from HIP events on the kernel's stream, against
             the 8 TB/s HBM peak; `traffic` from committed rocprofv3 counters
  first_run  one-shot cost: a new circuit of the distribution with its
             kernels built in the background (AUTO runs the interpreter
             meanwhile), the first pass of the headline circuit with the
             build in the foreground, the same circuit on the interpreter
             kernel, and the runs after which the build has paid for itself
  gate_per_pass  the same GPU, one sweep per gate: one- and two-qubit gates
             timed separately and projected onto the circuit's mix
  random34_c64  the 34-qubit complex64 state (same bytes) under the same
             protocol, with its own roofline
  streaming  in-place streaming rate of a plain one-gate sweep, n = 30..34
  sweep      the same circuit distribution at n = 30..32 (both dtypes), 33
             (complex64), n = 34 at k = 5 and 6, and the largest states that
             fit (35-qubit complex64, 34-qubit complex128; 256 GiB): one
             timed run each
  seed_spread  the headline distribution at 30 qubits complex128 over seeds
             0-4: median and spread of gates/s, pass rate and part count
  multilevel the same circuits with the multi-level partition (first level
             bounded by the padded LDS tile, 14 qubits complex64 / 13
             complex128; second level = register stages)
  layered28  28 qubits, 40 layers (U3 on every qubit + CX matching),
             k = 6, complex64 and complex128: interpreter (PART_LDS) vs
             specialized kernels vs AUTO vs one sweep per gate
  dressed30  deep dense five-qubit parts (dressed two-qubit blocks, ~80
             gates per part), k = 5: gate-by-gate vs fused vs AUTO
  qft32      a 32-qubit QFT on a random basis state, k = 7:
             gate-by-gate (specialized) vs fused-unitary (matrix cores) vs
             AUTO, with the fused kernel's matrix-core roofline
  serving    p50/p99 latency (from each request's scheduled arrival) and
             circuits/s of a Poisson stream of 1,000 requests at 40/s, and a
             latency-against-load curve of 250 requests at 20, 80, 160/s
  accuracy   U^-1 U |0> against |0> on sampled amplitudes of the headline
             state (untimed)
  cpu_baseline  the oracle (numpy complex128, one thread) on a bounded
             sample, extrapolated to the headline size
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gates/s + HBM GB/s per part-pass at n=30..34; p50/p99 latency in serving loop"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}  # dense FP32 / FP64 matrix cores
PROFILE_DIR = os.path.join(ROOT, "profiles")


def inverse_gates(gates):
    """The circuit's inverse: gates in reverse order, each inverted (the
    headline's kinds and the other parametrised ones)."""
    out = []
    for g in reversed(gates):
        name, p = g[0], tuple(g[3])
        if name in ("h", "x", "y", "z", "cx", "cz", "swap"):
            out.append(g)
        elif name in ("rx", "ry", "rz", "p", "cp"):
            out.append((name, g[1], g[2], (-p[0],)))
        elif name == "u3":
            out.append((name, g[1], g[2], (-p[0], -p[2], -p[1])))
        else:
            raise ValueError(f"no inverse for {name}")
    return out


def part_pass_bytes(n: int, dtype: str) -> int:
    """Algorithmic HBM bytes of one part-pass: every amplitude read and written once."""
    return 2 * (1 << n) * (8 if dtype == "c64" else 16)


def spec_kernel_hash(plan, dtype: str) -> str:
    """Identity of the specialized part kernels a plan runs: the generated
    source of every part plus the launcher that sizes their grids."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2205_06973_amd", "csrc", "specialize.cpp"), "rb") as fh:
        h.update(fh.read())
    for i in range(plan.num_parts):
        h.update(plan.part_source(i, dtype).encode())
    return h.hexdigest()[:16]


def committed_traffic(n: int, dtype: str, k: int, khash: str):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary, if it
    was taken on these very kernels (same generated sources) and workload."""
    path = os.path.join(PROFILE_DIR, "part_pass_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    rec = d.get("workloads", {}).get(f"n{n}_{dtype}_k{k}")
    if not rec or rec.get("kernel_hash") != khash:
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(n_target: int, seed: int, dtype: str, budget_s: float = 20.0, n_cpu: int = 28) -> dict:
    """The oracle as it stands, one host thread, on the first gates of the same
    circuit distribution at n_cpu qubits (complex128, the oracle's only
    precision); per-gate time scaled by 2^(n_target-n_cpu).  The oracle cannot
    hold the target state on the host in the time allowed (2^33 complex128
    amplitudes are 128 GiB), so the figure is extrapolated and says so."""
    from threadpoolctl import threadpool_limits

    from oracle import statevector as sv  # test infrastructure: this leg only
    from paper_2205_06973_amd import workloads as wl
    _, gates = wl.random34(seed, n=n_cpu)
    psi = sv.basis_state(n_cpu, 0)
    done = 0
    # elementwise numpy only; the BLAS pool is pinned to one thread regardless
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while done < len(gates):
            sv.apply_gate(psi, gates[done])
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    per_gate = dt / done
    scale = 2.0 ** (n_target - n_cpu)
    return {
        "value": 1.0 / (per_gate * scale), "unit": "gates/s", "cores": 1,
        "kind": "oracle, extrapolated",
        "sample": (f"numpy complex128 oracle, 1 thread, first {done} gates of the same "
                   f"distribution at n={n_cpu} ({dt:.1f} s); per-gate time x2^{n_target - n_cpu} "
                   f"to n={n_target} (the GPU state is {dtype})"),
        "extrapolated_from_n": n_cpu,
        # the oracle's own sweep rate at the sampled size (read + write of
        # every complex128 amplitude per gate)
        "oracle_GBps": 2 * (1 << n_cpu) * 16 / per_gate / 1e9,
        "host_cpus": len(os.sched_getaffinity(0)),
    }


def timed_plan(st, plan, stream, steps=1, mode="part_spec"):
    """Seconds of `steps` whole-plan runs (one warm run first), HIP events on the state's stream."""
    import torch
    st.simulate(plan, mode)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        st.simulate(plan, mode)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def run_sweep(args, buf, stream, log):
    """The headline circuit distribution over n = 30..35, k = 5..7 and both dtypes
    (the 33-qubit complex128 and 34-qubit complex64 k = 7 cases are the
    headline runs themselves)."""
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    cases = [(30, "c64", 7), (31, "c64", 7), (32, "c64", 7), (33, "c64", 7),
             (34, "c64", 5), (34, "c64", 6),
             (30, "c128", 7), (31, "c128", 7), (32, "c128", 7),
             (35, "c64", 7), (34, "c128", 7)]  # the last two: 256 GiB states
    rows = []
    for n, dt, k in cases:
        amp = 8 if dt == "c64" else 16
        if (1 << n) * amp > buf.numel() * buf.element_size():
            continue
        import torch
        view = buf.view(torch.uint8)[: (1 << n) * amp].view(
            torch.complex64 if dt == "c64" else torch.complex128)
        st = hisv.State.wrap_tensor(view, stream)
        st.set_basis(0)
        _, gates = wl.random34(args.seed, n=n, num_gates=args.gates)
        plan = hisv.Plan.partition(hisv.Circuit(n, gates), k, args.strategy, seed=args.seed,
                                   trials=args.trials)
        plan.specialize(dt)
        sec = timed_plan(st, plan, stream)
        norm = st.norm()
        st.close()
        P = plan.num_parts
        gbs = part_pass_bytes(n, dt) * P / sec / 1e9
        row = {"n": n, "dtype": dt, "k": k, "parts": P, "gates_per_s": len(gates) / sec,
               "ms_per_circuit": sec * 1e3, "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
               "norm_after": norm}
        log(f"[bench] sweep {row}")
        if not abs(norm - 1.0) < 1e-3:
            raise RuntimeError(f"norm drift in sweep case {row}")
        rows.append(row)
    return rows


def run_seed_spread(args, buf, stream, log, n=30, dt="c128", k=7, seeds=(0, 1, 2, 3, 4)):
    """The headline distribution at 30 qubits, complex128, over five seeds:
    median and spread of the per-circuit rate and part count."""
    import statistics
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    amp = 8 if dt == "c64" else 16
    view = buf.view(torch.uint8)[: (1 << n) * amp].view(torch.complex64 if dt == "c64" else torch.complex128)
    st = hisv.State.wrap_tensor(view, stream)
    rows = []
    for sd in seeds:
        st.set_basis(0)
        _, gates = wl.random34(sd, n=n, num_gates=args.gates)
        plan = hisv.Plan.partition(hisv.Circuit(n, gates), k, args.strategy, seed=sd, trials=args.trials)
        plan.specialize(dt)
        sec = timed_plan(st, plan, stream)
        gbs = part_pass_bytes(n, dt) * plan.num_parts / sec / 1e9
        rows.append({"seed": sd, "parts": plan.num_parts, "gates_per_s": len(gates) / sec,
                     "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS})
    st.close()
    g = [r["gates_per_s"] for r in rows]
    f = [r["frac"] for r in rows]
    out = {"n": n, "dtype": dt, "k": k, "seeds": list(seeds), "rows": rows,
           "gates_per_s_median": statistics.median(g), "gates_per_s_min": min(g), "gates_per_s_max": max(g),
           "frac_median": statistics.median(f), "frac_min": min(f), "frac_max": max(f),
           "parts": [r["parts"] for r in rows]}
    log(f"[bench] seed spread {out['gates_per_s_median']:.1f} gates/s median "
        f"({out['gates_per_s_min']:.1f}-{out['gates_per_s_max']:.1f}), parts {out['parts']}")
    return out


def run_multilevel(args, buf, stream, log):
    """Multi-level plans (Sec. IV.B): level-1 parts fill the padded LDS tile."""
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    rows = []
    s = args.strategy
    cases = [("random34", 34, "c64", s), ("random33", 33, "c128", s), ("qft32", 32, "c64", s)]
    for name, n, dt, strat in cases:
        amp = 8 if dt == "c64" else 16
        if (1 << n) * amp > buf.numel() * buf.element_size():
            continue
        view = buf.view(torch.uint8)[: (1 << n) * amp].view(
            torch.complex64 if dt == "c64" else torch.complex128)
        st = hisv.State.wrap_tensor(view, stream)
        st.set_basis(0)
        gates = wl.qft_circuit(n) if name == "qft32" else wl.random34(args.seed, n=n, num_gates=args.gates)[1]
        plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), strategy=strat, dtype=dt,
                                              seed=args.seed, trials=args.trials)
        plan.specialize(dt)
        sec = timed_plan(st, plan, stream)
        norm = st.norm()
        st.close()
        P = plan.num_parts
        gbs = part_pass_bytes(n, dt) * P / sec / 1e9
        row = {"workload": name, "n": n, "dtype": dt, "strategy": strat, "tile_qubits": plan.k,
               "pad_qubits": 6, "parts": P, "gates": len(gates), "gates_per_s": len(gates) / sec,
               "ms_per_circuit": sec * 1e3, "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
               "norm_after": norm}
        log(f"[bench] multilevel {row}")
        if not abs(norm - 1.0) < 1e-3:
            raise RuntimeError(f"norm drift in multi-level case {row}")
        rows.append(row)
    return rows


def run_layered(args, buf, stream, log):
    """28-qubit layered circuit (40 layers of U3 on every qubit + CX on a
    random perfect matching, 1,680 gates), DFS k = 6, complex64 and
    complex128: the gate-by-gate interpreter (PART_LDS), the specialized
    kernels (PART_SPEC), AUTO, and one sweep per gate."""
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    n, gates = wl.layered28(args.seed)
    k = 6
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), k, args.strategy, seed=args.seed,
                               trials=args.trials)
    P, G = plan.num_parts, len(gates)
    rows = []
    for dt in ("c64", "c128"):
        nbytes = (1 << n) * (8 if dt == "c64" else 16)
        view = buf.view(torch.uint8)[:nbytes].view(torch.complex64 if dt == "c64" else torch.complex128)
        st = hisv.State.wrap_tensor(view, stream)
        plan.specialize(dt)
        row = {"workload": "layered28", "n": n, "dtype": dt, "k": k, "strategy": args.strategy,
               "parts": P, "gates": G, "passes_saved": G / P}
        for mode in ("part_lds", "part_spec", "auto"):
            st.set_basis(0)
            sec = timed_plan(st, plan, stream, steps=3, mode=mode)
            gbs = part_pass_bytes(n, dt) * P / sec / 1e9
            row[mode] = {"gates_per_s": G / sec, "ms_per_circuit": sec * 1e3,
                         "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS, "norm_after": st.norm()}
            if not abs(row[mode]["norm_after"] - 1.0) < 1e-3:
                raise RuntimeError(f"norm drift in layered case {dt} {mode}")
        circ = hisv.Circuit(n, gates)
        st.simulate_gate_per_pass(circ)  # warm
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        st.simulate_gate_per_pass(circ)
        e1.record(stream)
        torch.cuda.synchronize()
        gpp = G / (e0.elapsed_time(e1) / 1e3)
        row["gate_per_pass_gates_per_s"] = gpp
        row["speedup_part_lds"] = row["part_lds"]["gates_per_s"] / gpp
        row["speedup_part_spec"] = row["part_spec"]["gates_per_s"] / gpp
        st.close()
        log(f"[bench] layered28 {row}")
        rows.append(row)
    return rows


def run_dressed(args, buf, stream, log):
    """Deep, dense five-qubit parts: dressed two-qubit blocks (U3 on both
    qubits, a CX / CZ / CP / SWAP, U3 again) drawn from a five-qubit window
    that moves up one qubit every 16 blocks; 600 blocks = 3,000 gates on 30
    qubits, k = 5 (about 80 gates per part).  Gate-by-gate (specialized) vs
    the fused dense unitary (matrix cores) vs AUTO, both dtypes."""
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    n, k = 30, 5
    gates = wl.dressed_pairs_circuit(n, 600, seed=3, span=5, dwell=16)
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), k, args.strategy, seed=args.seed,
                               trials=args.trials)
    P, G = plan.num_parts, len(gates)
    rows = []
    for dt in ("c64", "c128"):
        nbytes = (1 << n) * (8 if dt == "c64" else 16)
        view = buf.view(torch.uint8)[:nbytes].view(torch.complex64 if dt == "c64" else torch.complex128)
        st = hisv.State.wrap_tensor(view, stream)
        plan.specialize(dt)
        row = {"workload": "dressed30", "n": n, "dtype": dt, "k": k, "strategy": args.strategy,
               "parts": P, "gates": G, "auto_fused_parts": int(plan.auto_choice(dt).sum())}
        for mode in ("part_spec", "part_fused", "auto"):
            st.set_basis(0)
            sec = timed_plan(st, plan, stream, steps=2, mode=mode)
            gbs = part_pass_bytes(n, dt) * P / sec / 1e9
            row[mode] = {"gates_per_s": G / sec, "ms_per_circuit": sec * 1e3,
                         "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS, "norm_after": st.norm()}
            if not abs(row[mode]["norm_after"] - 1.0) < 1e-3:
                raise RuntimeError(f"norm drift in dressed case {dt} {mode}")
        row["speedup_auto_over_part_spec"] = (row["part_spec"]["ms_per_circuit"]
                                              / row["auto"]["ms_per_circuit"])
        st.close()
        log(f"[bench] dressed30 {row}")
        rows.append(row)
    return rows


def run_qft(buf, stream, log, strategy="closure", trials=16):
    """32-qubit QFT (H + controlled-phase ladder + swaps) on a random basis
    state, dagP k = 7: gate-by-gate specialized kernels (a) vs the fused dense
    unitary on matrix cores (b) vs AUTO; sampled amplitudes against the closed
    form e^{2 pi i x y / 2^n} / 2^{n/2}."""
    import numpy as np
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    n, dt = 32, "c64"
    if (1 << n) * 8 > buf.numel() * buf.element_size():
        return None
    view = buf.view(torch.uint8)[: (1 << n) * 8].view(torch.complex64)
    st = hisv.State.wrap_tensor(view, stream)
    gates = wl.qft_circuit(n)
    x = wl.random_basis_index(n, 3)
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), 7, strategy, seed=0, trials=trials)
    plan.specialize(dt)
    P = plan.num_parts
    idx = np.unique(np.random.default_rng(1).integers(0, 1 << n, 4096, dtype=np.uint64))
    want = np.exp(2j * np.pi * ((int(x) * idx.astype(object)) % (1 << n)).astype(np.float64)
                  / (1 << n)) / 2 ** (n / 2)
    out = {"n": n, "dtype": dt, "k": 7, "strategy": strategy, "parts": P, "gates": len(gates)}
    for mode in ("part_spec", "part_fused", "auto"):
        st.set_basis(int(x))
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(P + 1)]
        ev[0].record(stream)
        for i in range(P):
            st.simulate_part(plan, i, mode)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(P)]
        err = float(np.max(np.abs(st.amplitudes_at(idx) - want)))
        ms = sum(per)
        row = {"ms_per_circuit": ms, "gates_per_s": len(gates) / ms * 1e3,
               "max_abs_err_sampled": err}
        if mode == "part_fused":
            w7 = [per[i] for i in range(P) if len(plan.part_unitary(i)[0]) == 7]
            if w7:
                avg = sum(w7) / len(w7)
                flops = 8.0 * 128 * (1 << n)  # 8 flops per complex multiply-add, 2^w per amplitude
                tf = flops / (avg / 1e3) / 1e12
                row["w7_parts"] = len(w7)
                row["mfma_roofline"] = {"bound": "mfma", "achieved": tf, "peak": MFMA_PEAK_TFLOPS[dt],
                                        "unit": "TFLOP/s", "frac": tf / MFMA_PEAK_TFLOPS[dt],
                                        "avg_launch_ms": avg}
        out[mode] = row
        log(f"[bench] qft32 {mode}: {row}")
    st.close()
    out["speedup_gate_by_gate_over_fused"] = out["part_fused"]["ms_per_circuit"] / out["part_spec"]["ms_per_circuit"]
    return out


def whole_path(args, n, dt, k, gates, view, stream, steps, warmup, log):
    """Time `steps` passes of the whole path on one state (after `warmup`).

    A pass ingests the gate list, partitions it, compiles it (specialized
    kernels come from the kernel cache once built), applies every part and
    reads the FP64 norm back.  The very first pass of a circuit also builds
    its kernels: it is timed on its own (`first_run`) next to the same
    circuit on the interpreter kernel, which needs no build."""
    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    G = len(gates)
    st = hisv.State.wrap_tensor(view, stream)
    st.set_basis(0)
    mode = args.mode

    def step(events=None, run_mode=mode):
        circ = hisv.Circuit(n, gates)
        plan = hisv.Plan.partition(circ, k, args.strategy, seed=args.seed, trials=args.trials)
        if run_mode == "part_spec":
            plan.specialize(dt)
        if events is not None:
            events[0].record(stream)
        st.simulate(plan, run_mode)
        if events is not None:
            events[1].record(stream)
        return plan, st.norm()

    # one-shot cost.  A new circuit of the same distribution with its kernels
    # built in the background: AUTO runs the interpreter until they are
    # ready (the build is waited for afterwards, untimed).  Then the first
    # pass of this circuit with the build in the foreground, and the same
    # circuit on the interpreter kernel.
    first = {}
    if mode == "part_spec":
        _, other = wl.random34(args.seed + 1, n=n, num_gates=G)
        torch.cuda.synchronize()
        t = time.perf_counter()
        oplan = hisv.Plan.partition(hisv.Circuit(n, other), k, args.strategy, seed=args.seed,
                                    trials=args.trials)
        oplan.specialize_async(dt)
        st.simulate(oplan, "auto")
        norm = st.norm()
        first["background_build_wall_s"] = time.perf_counter() - t
        oplan.specialize_wait(dt)
        if not abs(norm - 1.0) < 1e-3:
            raise RuntimeError(f"norm {norm} after the background-build pass")
        st.set_basis(0)
    for label, m in (("wall_s", mode), ("interpreter_wall_s", "part_lds")):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan, norm = step(run_mode=m)
        torch.cuda.synchronize()
        first[label] = time.perf_counter() - t
        if not abs(norm - 1.0) < 1e-3:
            raise RuntimeError(f"norm {norm} after the first {m} pass")
    P = plan.num_parts
    log(f"[bench] n={n} {dt} G={G} k={k} {args.strategy}: {P} parts; first pass "
        f"{first['wall_s']:.2f} s ({mode}, kernel build included), "
        f"{first['interpreter_wall_s']:.2f} s (part_lds)")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plan, norm = step(ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = sum(a.elapsed_time(b) for a, b in ev)
    log(f"[bench] timed {steps} steps: wall {wall:.3f} s, part kernels (events) {gpu_ms:.1f} ms")
    if not abs(norm - 1.0) < 1e-3:
        # a unitary circuit keeps the norm: anything else is a wrong result
        raise RuntimeError(f"norm after the timed steps is {norm}, not 1")
    launches = steps * P
    avg_launch_s = gpu_ms / 1e3 / launches
    bpl = part_pass_bytes(n, dt)
    achieved = bpl / avg_launch_s / 1e9
    khash = spec_kernel_hash(plan, dt) if mode == "part_spec" else None
    traffic = committed_traffic(n, dt, k, khash) if khash else None
    warm_s = wall / steps
    first["gates_per_s"] = G / first["wall_s"]
    first["interpreter_gates_per_s"] = G / first["interpreter_wall_s"]
    if "background_build_wall_s" in first:
        first["background_build_gates_per_s"] = G / first["background_build_wall_s"]
    # runs of the same circuit after which the kernel build has paid for itself
    gain = first["interpreter_wall_s"] - warm_s
    first["break_even_runs"] = ((first["wall_s"] - warm_s) / gain) if gain > 0 else None
    res = {
        "value": G * steps / wall, "ms_per_step": warm_s * 1e3, "plan": plan, "norm": norm,
        "parts": P, "first_run": first, "gpu_ms": gpu_ms,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": {"part_spec": "part_pass_spec", "part_lds": "part_pass_kernel",
                       "auto": "part_pass_kernel+fused_pass_kernel"}[mode],
            "bytes_per_launch": bpl,
            "avg_launch_us": avg_launch_s * 1e6, "launches": launches, "kernel_hash": khash,
        },
        "state": st,
    }
    return res


def round_trip_error(args, st, plan, n, k, gates):
    """U then U^-1 from |0> must give |0> again (untimed; the inverse runs on
    the interpreter: no second kernel build)."""
    import numpy as np
    from paper_2205_06973_amd import hisv
    st.set_basis(0)
    st.simulate(plan, args.mode)
    inv = hisv.Plan.partition(hisv.Circuit(n, inverse_gates(gates)), k, args.strategy,
                              seed=args.seed, trials=64)
    st.simulate(inv, "part_lds")
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(4096, dtype=np.uint64),
                                    rng.integers(0, 1 << n, 1 << 14, dtype=np.uint64),
                                    np.arange((1 << n) - 4096, 1 << n, dtype=np.uint64)]))
    amp = st.amplitudes_at(idx)
    return idx.size, float(np.max(np.abs(amp - (idx == 0))))


def gate_per_pass(st, n, dt, gates, stream, count, part_kernel_s):
    """One sweep per gate on the same state, timed separately for one- and
    two-qubit gates (a two-qubit sweep leaves a quarter of the amplitudes
    alone), then projected onto the whole circuit's mix of the two."""
    import torch
    from paper_2205_06973_amd import hisv
    one = [g for g in gates if g[2] < 0][:count]
    two = [g for g in gates if g[2] >= 0][:count]
    per = {}
    for name, sub in (("1q", one), ("2q", two)):
        circ = hisv.Circuit(n, sub)
        st.simulate_gate_per_pass(circ)  # warm
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        st.simulate_gate_per_pass(circ)
        e1.record(stream)
        torch.cuda.synchronize()
        per[name] = e0.elapsed_time(e1) / 1e3 / len(sub)
    n1 = sum(1 for g in gates if g[2] < 0)
    n2 = len(gates) - n1
    circuit_s = n1 * per["1q"] + n2 * per["2q"]
    bpl = part_pass_bytes(n, dt)
    return {
        "gates_timed": {"1q": len(one), "2q": len(two)},
        "ms_per_gate": {"1q": per["1q"] * 1e3, "2q": per["2q"] * 1e3},
        "pass_GBps_1q": bpl / per["1q"] / 1e9,
        "circuit_gates": {"1q": n1, "2q": n2},
        "gates_per_s": len(gates) / circuit_s,
        # like for like: kernel time of the partitioned path (HIP events)
        # against the projected kernel time of one sweep per gate
        "speedup_partitioned_kernels": circuit_s / part_kernel_s,
    }


def streaming_ceiling(buf, stream, log, cases):
    """In-place streaming rate of the plainest full-state sweep: one
    single-qubit gate (H on the lowest qubit) per pass, per size."""
    import torch
    from paper_2205_06973_amd import hisv
    rows = []
    for n, dt in cases:
        amp = 8 if dt == "c64" else 16
        if (1 << n) * amp > buf.numel() * buf.element_size():
            continue
        view = buf.view(torch.uint8)[: (1 << n) * amp].view(
            torch.complex64 if dt == "c64" else torch.complex128)
        st = hisv.State.wrap_tensor(view, stream)
        st.set_basis(0)
        circ = hisv.Circuit(n, [("h", 0, -1, ())] * 8)
        st.simulate_gate_per_pass(circ)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        st.simulate_gate_per_pass(circ)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / 8
        gbs = part_pass_bytes(n, dt) / sec / 1e9
        rows.append({"n": n, "dtype": dt, "ms_per_pass": sec * 1e3, "pass_GBps": gbs,
                     "frac": gbs / HBM_PEAK_GBS})
        st.close()
        log(f"[bench] streaming {rows[-1]}")
    return rows


def tile_scan(buf, stream, log, sizes=(28, 30, 32, 34), reps=8):
    """One part whose tile is a single contiguous run (H twice on qubits
    6-12, tile = qubits 0-12, complex64), specialized, at several state
    sizes: the part kernel's rate without scattered runs or re-layouts."""
    import torch
    from paper_2205_06973_amd import hisv
    rows = []
    for n in sizes:
        if (1 << n) * 8 > buf.numel() * buf.element_size():
            continue
        gates = [("h", q, -1, ()) for q in range(6, 13)] * 2
        plan = hisv.Plan.partition(hisv.Circuit(n, gates), 7, "greedy", seed=0, trials=4)
        plan.specialize("c64")
        view = buf.view(torch.uint8)[: (1 << n) * 8].view(torch.complex64)
        st = hisv.State.wrap_tensor(view, stream)
        st.set_basis(0)
        sec = timed_plan(st, plan, stream, steps=reps)
        gbs = part_pass_bytes(n, "c64") / sec / 1e9
        rows.append({"n": n, "dtype": "c64", "parts": plan.num_parts, "ms_per_pass": sec * 1e3,
                     "pass_GBps": gbs, "frac": gbs / HBM_PEAK_GBS})
        st.close()
        log(f"[bench] tile scan {rows[-1]}")
    return rows


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=33)
    ap.add_argument("--gates", type=int, default=1000)
    ap.add_argument("--k", type=int, default=7)
    ap.add_argument("--dtype", default="c128", choices=["c64", "c128"])
    ap.add_argument("--strategy", default="closure", choices=["nat", "dfs", "dagp", "greedy", "closure"])
    ap.add_argument("--trials", type=int, default=None,
                    help="orders (DFS), tie-break draws (greedy) or beam width (closure) per partition "
                         "(default: 16 for closure, else 256)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="part_spec", choices=["part_lds", "part_spec", "auto"])
    ap.add_argument("--gpp-gates", type=int, default=24,
                    help="one- and two-qubit gates each timed on the gate-per-pass baseline (0 = skip)")
    ap.add_argument("--c64-steps", type=int, default=2,
                    help="timed steps of the 34-qubit complex64 companion run (0 = skip)")
    ap.add_argument("--serving", type=int, default=1000, help="serving requests (0 = skip)")
    ap.add_argument("--serving-rate", type=float, default=40.0, help="arrivals per second")
    ap.add_argument("--serving-curve", type=float, nargs="*", default=[20.0, 80.0, 160.0],
                    help="further arrival rates, each with --serving-curve-requests requests")
    ap.add_argument("--serving-curve-requests", type=int, default=250)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="layout knob passed to hs_tune before the plan is compiled")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run the plain copy kernel on this many GiB (counter calibration)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the n / k / dtype sweep")
    ap.add_argument("--no-streaming", action="store_true", help="skip the streaming-rate probe")
    ap.add_argument("--no-qft", action="store_true", help="skip the 32-qubit QFT comparison")
    ap.add_argument("--no-multilevel", action="store_true", help="skip the multi-level partition runs")
    ap.add_argument("--no-layered", action="store_true", help="skip the 28-qubit layered circuit runs")
    ap.add_argument("--no-dressed", action="store_true", help="skip the dense five-qubit-part runs")
    ap.add_argument("--layered-only", action="store_true",
                    help="run only the 28-qubit layered section (for profiling)")
    ap.add_argument("--qft-only", action="store_true",
                    help="run only the 32-qubit QFT comparison (for kernel profiles)")
    ap.add_argument("--streaming-only", action="store_true",
                    help="run only the streaming-rate probe (for profiles)")
    ap.add_argument("--tile-scan-only", action="store_true",
                    help="run only the contiguous-tile part at 28-34 qubits (for profiles)")
    ap.add_argument("--dressed-only", action="store_true",
                    help="run only the dense five-qubit-part comparison (for kernel profiles)")
    args = ap.parse_args()
    if args.trials is None:
        args.trials = 16 if args.strategy == "closure" else 256

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        return 2

    import torch
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    for kv in args.tune:
        key, val = kv.split("=")
        hisv.hs_tune(key, int(val))
    stream = torch.cuda.Stream()
    stream_cases = [(30, "c64"), (31, "c64"), (32, "c64"), (33, "c64"), (34, "c64"),
                    (30, "c128"), (31, "c128"), (32, "c128"), (33, "c128")]
    if args.layered_only:
        with torch.cuda.stream(stream):
            lbuf = torch.empty(1 << 28, dtype=torch.complex128, device="cuda")
        print(json.dumps({"layered28": run_layered(args, lbuf, stream, log)}), flush=True)
        return 0
    if args.qft_only:
        with torch.cuda.stream(stream):
            qbuf = torch.empty(1 << 32, dtype=torch.complex64, device="cuda")
        print(json.dumps({"qft32": run_qft(qbuf, stream, log, args.strategy, args.trials)}), flush=True)
        return 0
    if args.tile_scan_only:
        with torch.cuda.stream(stream):
            tbuf = torch.empty(1 << 34, dtype=torch.complex64, device="cuda")
        print(json.dumps({"streaming": tile_scan(tbuf, stream, log)}), flush=True)
        return 0
    if args.dressed_only:
        with torch.cuda.stream(stream):
            dbuf = torch.empty(1 << 30, dtype=torch.complex128, device="cuda")
        out = {"dressed30": run_dressed(args, dbuf, stream, log)}
        del dbuf
        torch.cuda.empty_cache()
        if args.copy_probe_gib > 0:
            nbytes = int(args.copy_probe_gib * 2**30) // 16 * 16
            a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            b = torch.empty_like(a)
            hisv.hs_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, stream)
            torch.cuda.synchronize()
            out["copy_probe_bytes"] = nbytes
        print(json.dumps(out), flush=True)
        return 0
    if args.streaming_only:
        with torch.cuda.stream(stream):
            sbuf = torch.empty(1 << 34, dtype=torch.complex64, device="cuda")
        print(json.dumps({"streaming": streaming_ceiling(sbuf, stream, log, stream_cases)}), flush=True)
        return 0

    n, G, dt = args.n, args.gates, args.dtype
    _, gates = wl.random34(args.seed, n=n, num_gates=G)
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    with torch.cuda.stream(stream):
        buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    head = whole_path(args, n, dt, args.k, gates, buf, stream, args.steps, args.warmup, log)
    st, plan, P = head["state"], head["plan"], head["parts"]
    bpl = part_pass_bytes(n, dt)
    state_name = "complex64" if dt == "c64" else "complex128"
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dt == "c64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"random{n}: {n}-qubit random circuit, {G} gates uniform over "
                         f"{{H,RZ,RX,CX,CZ}}, {state_name} state ({bpl // 2 / 2**30:.0f} GiB), "
                         f"{args.strategy.upper()} partition k={args.k}"),
            "n": n, "gates": G, "k": args.k, "parts": P, "strategy": args.strategy,
            "state": state_name, "mode": args.mode, "passes_saved": G / P,
        },
        "roofline": head["roofline"],
        "first_run": head["first_run"],
        "norm_after": head["norm"],
    }
    cnt, err = round_trip_error(args, st, plan, n, args.k, gates)
    out["accuracy"] = {
        "check": f"U^-1 U |0> against |0> on {cnt} amplitudes (first and last 4096, 2^14 random)",
        "max_abs_err": err, "tolerance": 2e-5 if dt == "c64" else 1e-12,
    }
    log(f"[bench] round trip max |d| = {err:.3e}")
    if args.gpp_gates > 0:
        gpp = gate_per_pass(st, n, dt, gates, stream, args.gpp_gates,
                            head["gpu_ms"] / 1e3 / args.steps)
        gpp["passes_saved"] = G / P
        gpp["speedup_partitioned"] = out["value"] / gpp["gates_per_s"]
        out["gate_per_pass"] = gpp
        log(f"[bench] gate-per-pass: {gpp}")
    st.close()

    if args.c64_steps > 0 and dt == "c128" and n == 33:
        # the same bytes as a 34-qubit complex64 state: that workload on the
        # same buffer, same protocol
        view = buf.view(torch.complex64)
        _, g34 = wl.random34(args.seed, n=34, num_gates=G)
        r = whole_path(args, 34, "c64", args.k, g34, view, stream, args.c64_steps, 1, log)
        r["state"].close()
        out["random34_c64"] = {
            "workload": (f"random34: 34-qubit random circuit, {G} gates, complex64 state (128 GiB), "
                         f"{args.strategy.upper()} partition k={args.k}"),
            "dtype": "f32", "gates_per_s": r["value"], "ms_per_step": r["ms_per_step"],
            "steps": args.c64_steps, "parts": r["parts"], "roofline": r["roofline"],
            "first_run": r["first_run"], "norm_after": r["norm"],
        }
        log(f"[bench] random34 c64: {r['value']:.1f} gates/s, frac {r['roofline']['frac']:.3f}")
        del view, r  # the view shares the buffer's memory
    del head, st

    if not (args.no_sweep and args.no_multilevel and args.no_qft and args.no_layered
            and args.no_streaming and args.no_dressed):
        # the extra sections share one buffer: 256 GiB (a 35-qubit complex64 or
        # 34-qubit complex128 state) when the device has room, else the
        # headline's
        if torch.cuda.mem_get_info()[0] + buf.numel() * buf.element_size() >= (256 << 30) + (4 << 30):
            del buf
            torch.cuda.empty_cache()
            with torch.cuda.stream(stream):
                buf = torch.empty(1 << 35, dtype=torch.complex64, device="cuda")
        if not args.no_streaming:
            out["streaming"] = streaming_ceiling(buf, stream, log, stream_cases)
        if not args.no_sweep:
            out["sweep"] = run_sweep(args, buf, stream, log)
            out["seed_spread"] = run_seed_spread(args, buf, stream, log)
        if not args.no_multilevel:
            out["multilevel"] = run_multilevel(args, buf, stream, log)
        if not args.no_layered:
            out["layered28"] = run_layered(args, buf, stream, log)
        if not args.no_dressed:
            out["dressed30"] = run_dressed(args, buf, stream, log)
        if not args.no_qft:
            out["qft32"] = run_qft(buf, stream, log, args.strategy, args.trials)
    del buf
    torch.cuda.empty_cache()

    if args.copy_probe_gib > 0:
        nbytes = int(args.copy_probe_gib * 2**30) // 16 * 16
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        hisv.hs_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, stream)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
        del a, b
        torch.cuda.empty_cache()

    if args.serving > 0:
        from paper_2205_06973_amd import serving
        reqs = wl.serving_stream(args.serving, args.serving_rate, seed=args.seed)
        res = serving.run_stream(reqs)
        out["serving"] = serving.summarize(res, len(reqs))
        out["serving"].update({"arrival_rate_per_s": args.serving_rate,
                               "peak_inflight": res["stats"]["peak_inflight"],
                               "peak_admitted_GiB": res["stats"]["peak_bytes"] / 2**30})
        log(f"[bench] serving: {out['serving']}")
        # latency against load: shorter streams at other arrival rates
        curve = []
        for rate in args.serving_curve:
            creqs = wl.serving_stream(args.serving_curve_requests, rate, seed=args.seed + 1)
            cres = serving.run_stream(creqs)
            row = serving.summarize(cres, len(creqs))
            curve.append({"arrival_rate_per_s": rate, "requests": len(creqs), "p50_ms": row["p50_ms"],
                          "p99_ms": row["p99_ms"], "circuits_per_s": row["circuits_per_s"],
                          "host_share": row["host_share"]})
            log(f"[bench] serving curve {curve[-1]}")
        if curve:
            out["serving"]["curve"] = curve

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.seed, dt)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3g} gates/s")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
