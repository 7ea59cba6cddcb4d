#!/usr/bin/env python3
"""Benchmark of the partitioned state-vector hot path on one MI355X.

A step is one pass of the whole path over one circuit: the gate list is
loaded, partitioned (greedy ready-set partitioner; --strategy picks Nat,
DFS or dagP of Sec. IV.B instead) and compiled (the specialized part
kernels come from the kernel cache after the warmup), every part is applied
as one in-place Gather-Execute-Scatter sweep of a state resident in HBM
(Alg. 1), and the FP64 norm is read back.  Default workload: a 34-qubit random
circuit of 1,000 gates drawn uniformly from {H, RZ, RX, CX, CZ}, complex64
state (128 GiB), acyclic partition with at most k qubits per part.

Prints ONE JSON line on stdout:
  value      gates/s over the timed steps (wall clock, synchronized; host
             ingest, partition and compile included)
  roofline   the part-pass kernel: algorithmic bytes per launch (read + write
             every amplitude once: 2 * 2^n * bytes/amplitude) / the average
             launch duration from HIP events on the kernel's stream, against
             the 8 TB/s HBM peak; `traffic` from committed rocprofv3 counters
  gate_per_pass  the same GPU, one sweep per gate, on the circuit's first gates
  serving    p50/p99 latency and circuits/s of a short Poisson request stream
  sweep      the same circuit distribution at n = 30..33 (k = 7), n = 34 at
             k = 5 and 6, a 33-qubit complex128 state, and the largest states
             that fit (35-qubit complex64, 34-qubit complex128; 256 GiB):
             one timed step each
  multilevel the same circuits with the multi-level partition (first level
             bounded by the padded LDS tile, 14 qubits complex64 / 13
             complex128; second level = register stages)
  layered28  28 qubits, 40 layers (U3 on every qubit + CX matching),
             k = 6, complex64 and complex128: interpreter (PART_LDS) vs
             specialized kernels vs AUTO vs one sweep per gate
  qft32      a 32-qubit QFT on a random basis state, k = 7:
             gate-by-gate (specialized) vs fused-unitary (matrix cores) vs
             AUTO, with the fused kernel's matrix-core roofline
  accuracy   U^-1 U |0> against |0> on sampled amplitudes of the headline
             state (untimed)
  cpu_baseline  the oracle (numpy complex128) on a bounded sample
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


def cpu_baseline(n_target: int, seed: int, budget_s: float = 12.0, n_cpu: int = 24) -> dict:
    """The oracle as it stands, one host thread, on the first gates of the same
    circuit distribution at n_cpu qubits; per-gate time scaled by 2^(n_target-n_cpu)."""
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
        "value": 1.0 / (per_gate * scale), "unit": "gates/s", "cores": 1, "kind": "oracle",
        "sample": (f"numpy complex128 oracle, 1 thread, first {done} gates of the same "
                   f"distribution at n={n_cpu} ({dt:.1f} s); per-gate time x2^{n_target - n_cpu} "
                   f"to n={n_target}"),
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
    """The headline circuit distribution over n = 30..34, k = 5..7 and both dtypes."""
    from paper_2205_06973_amd import hisv
    from paper_2205_06973_amd import workloads as wl
    cases = [(30, "c64", 7), (31, "c64", 7), (32, "c64", 7), (33, "c64", 7),
             (34, "c64", 5), (34, "c64", 6), (33, "c128", 7),
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


def run_qft(buf, stream, log, strategy="greedy", trials=256):
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=34)
    ap.add_argument("--gates", type=int, default=1000)
    ap.add_argument("--k", type=int, default=7)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--strategy", default="greedy", choices=["nat", "dfs", "dagp", "greedy"])
    ap.add_argument("--trials", type=int, default=256,
                    help="orders (DFS) or tie-break draws (greedy) tried per partition")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="part_spec", choices=["part_lds", "part_spec", "auto"])
    ap.add_argument("--gpp-gates", type=int, default=48,
                    help="gates timed on the gate-per-pass baseline (0 = skip)")
    ap.add_argument("--serving", type=int, default=120, help="serving requests (0 = skip)")
    ap.add_argument("--serving-rate", type=float, default=40.0, help="arrivals per second")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="layout knob passed to hs_tune before the plan is compiled")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run the plain copy kernel on this many GiB (counter calibration)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the n / k / dtype sweep")
    ap.add_argument("--no-qft", action="store_true", help="skip the 32-qubit QFT comparison")
    ap.add_argument("--no-multilevel", action="store_true", help="skip the multi-level partition runs")
    ap.add_argument("--no-layered", action="store_true", help="skip the 28-qubit layered circuit runs")
    ap.add_argument("--layered-only", action="store_true",
                    help="run only the 28-qubit layered section (for profiling)")
    ap.add_argument("--qft-only", action="store_true",
                    help="run only the 32-qubit QFT comparison (for kernel profiles)")
    args = ap.parse_args()

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
    if args.layered_only:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            lbuf = torch.empty(1 << 28, dtype=torch.complex128, device="cuda")
        print(json.dumps({"layered28": run_layered(args, lbuf, stream, log)}), flush=True)
        return 0
    if args.qft_only:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            qbuf = torch.empty(1 << 32, dtype=torch.complex64, device="cuda")
        print(json.dumps({"qft32": run_qft(qbuf, stream, log, args.strategy, args.trials)}), flush=True)
        return 0
    n, G = args.n, args.gates
    _, gates = wl.random34(args.seed, n=n, num_gates=G)
    stream = torch.cuda.Stream()
    tdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    with torch.cuda.stream(stream):
        buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    st = hisv.State.wrap_tensor(buf, stream)
    st.set_basis(0)

    def step(events=None):
        """One pass of the whole path: ingest the gate list, partition, compile
        (specialized kernels come from the kernel cache after the first step),
        apply every part, read the FP64 norm back."""
        circ = hisv.Circuit(n, gates)
        plan = hisv.Plan.partition(circ, args.k, args.strategy, seed=args.seed, trials=args.trials)
        if args.mode == "part_spec":
            plan.specialize(args.dtype)
        if events is not None:
            events[0].record(stream)
        st.simulate(plan, args.mode)
        if events is not None:
            events[1].record(stream)
        return plan, st.norm()

    t = time.perf_counter()
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), args.k, args.strategy, seed=args.seed,
                               trials=args.trials)
    part_ms = (time.perf_counter() - t) * 1e3
    P = plan.num_parts
    log(f"[bench] n={n} G={G} k={args.k} {args.strategy}: {P} parts ({part_ms:.1f} ms)")
    spec_s = 0.0
    if args.mode == "part_spec":
        t = time.perf_counter()
        plan.specialize(args.dtype)  # compiles and caches the part kernels
        spec_s = time.perf_counter() - t
        log(f"[bench] specialized {P} part kernels in {spec_s:.1f} s")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan, norm = step(ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = sum(a.elapsed_time(b) for a, b in ev)
    log(f"[bench] timed {args.steps} steps: wall {wall:.3f} s, part kernels (events) {gpu_ms:.1f} ms")
    if not abs(norm - 1.0) < 1e-3:
        # a unitary circuit keeps the norm: anything else is a wrong result
        log(f"[bench] ERROR: norm after the timed steps is {norm}, not 1")
        return 3

    launches = args.steps * P
    avg_launch_s = gpu_ms / 1e3 / launches
    bpl = part_pass_bytes(n, args.dtype)
    achieved = bpl / avg_launch_s / 1e9
    # the committed counters were taken on the specialized kernels
    khash = spec_kernel_hash(plan, args.dtype) if args.mode == "part_spec" else None
    traffic = committed_traffic(n, args.dtype, args.k, khash) if khash else None
    out = {
        "metric": METRIC,
        "value": G * args.steps / wall,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "c64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"random{n}: {n}-qubit random circuit, {G} gates uniform over "
                         f"{{H,RZ,RX,CX,CZ}}, {'complex64' if args.dtype == 'c64' else 'complex128'} "
                         f"state ({bpl // 2 / 2**30:.0f} GiB), {args.strategy.upper()} partition k={args.k}"),
            "n": n, "gates": G, "k": args.k, "parts": P, "strategy": args.strategy,
            "state": "complex64" if args.dtype == "c64" else "complex128", "mode": args.mode,
            "passes_saved": G / P, "specialize_s": spec_s,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": {"part_spec": "part_pass_spec", "part_lds": "part_pass_kernel",
                       "auto": "part_pass_kernel+fused_pass_kernel"}[args.mode],
            "bytes_per_launch": bpl,
            "avg_launch_us": avg_launch_s * 1e6, "launches": launches, "kernel_hash": khash,
        },
        "norm_after": norm,
    }

    # accuracy at full size, untimed: U then U^-1 from |0> must give |0> again
    # (the inverse runs on the interpreter: no second kernel build)
    import numpy as np
    st.set_basis(0)
    st.simulate(plan, args.mode)
    inv = hisv.Plan.partition(hisv.Circuit(n, inverse_gates(gates)), args.k, args.strategy,
                              seed=args.seed, trials=64)
    st.simulate(inv, "part_lds")
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(4096, dtype=np.uint64),
                                    rng.integers(0, 1 << n, 1 << 14, dtype=np.uint64),
                                    np.arange((1 << n) - 4096, 1 << n, dtype=np.uint64)]))
    amp = st.amplitudes_at(idx)
    err = float(np.max(np.abs(amp - (idx == 0))))
    out["accuracy"] = {
        "check": f"U^-1 U |0> against |0> on {idx.size} amplitudes (first and last 4096, "
                 f"2^14 random)",
        "max_abs_err": err, "tolerance": 2e-5 if args.dtype == "c64" else 1e-12,
    }
    log(f"[bench] round trip max |d| = {err:.3e}")

    if args.gpp_gates > 0:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        sub = hisv.Circuit(n, gates[:args.gpp_gates])
        st.simulate_gate_per_pass(sub)  # warm
        torch.cuda.synchronize()
        e0.record(stream)
        st.simulate_gate_per_pass(sub)
        e1.record(stream)
        torch.cuda.synchronize()
        gpp_s = e0.elapsed_time(e1) / 1e3
        gpp_rate = args.gpp_gates / gpp_s
        out["gate_per_pass"] = {
            "gates_timed": args.gpp_gates, "gates_per_s": gpp_rate,
            "pass_GBps": bpl / (gpp_s / args.gpp_gates) / 1e9,
            "speedup_partitioned": out["value"] / gpp_rate,
            # like for like: both sides' kernel time from HIP events
            "speedup_partitioned_kernels": (G * args.steps / (gpu_ms / 1e3)) / gpp_rate,
            "passes_saved": G / P,
            # a two-qubit sweep leaves the |00> amplitude of every quad alone
            # (3/4 of the state moves), so in HBM bytes the saving is smaller
            "traffic_passes_saved": (sum(1 for g in gates if g[2] < 0)
                                     + 0.75 * sum(1 for g in gates if g[2] >= 0)) / P,
        }
        log(f"[bench] gate-per-pass: {gpp_rate:.1f} gates/s")

    st.close()

    if not (args.no_sweep and args.no_multilevel and args.no_qft and args.no_layered):
        # the extra sections share one buffer: 256 GiB (a 35-qubit complex64 or
        # 34-qubit complex128 state) when the device has room, else the
        # headline's
        big = None
        if torch.cuda.mem_get_info()[0] + buf.numel() * buf.element_size() >= (256 << 30) + (4 << 30):
            del buf
            torch.cuda.empty_cache()
            with torch.cuda.stream(stream):
                big = torch.empty(1 << 35, dtype=torch.complex64, device="cuda")
            buf = big
        if not args.no_sweep:
            out["sweep"] = run_sweep(args, buf, stream, log)
        if not args.no_multilevel:
            out["multilevel"] = run_multilevel(args, buf, stream, log)
        if not args.no_layered:
            out["layered28"] = run_layered(args, buf, stream, log)
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
        lat, swall, stats, _ = serving.run_stream(reqs)
        out["serving"] = serving.summarize(lat, swall, len(reqs))
        out["serving"].update({"arrival_rate_per_s": args.serving_rate,
                               "peak_inflight": stats["peak_inflight"],
                               "peak_admitted_GiB": stats["peak_bytes"] / 2**30})
        log(f"[bench] serving: {out['serving']}")

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.seed)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3g} gates/s")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
