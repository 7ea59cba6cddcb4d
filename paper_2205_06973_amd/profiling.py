"""Turn rocprofv3 output into the committed kernel summaries under profiles/.

    python -m paper_2205_06973_amd.profiling stats  <stats.csv> <out.txt> "<command>" [--kernel-hash H]
    python -m paper_2205_06973_amd.profiling traffic <fetch.csv> <write.csv> <key> "<command>" \
        --copy-bytes B --kernel-hash H [--txt out.txt]
    python -m paper_2205_06973_amd.profiling mfma <counters.csv> <stats.csv> <out.txt> "<command>"
    python -m paper_2205_06973_amd.profiling valu <counters.csv> <stats.csv> <out.txt> "<command>"
    python -m paper_2205_06973_amd.profiling waits <counters.csv> <stats.csv> <out.txt> "<command>"
    python -m paper_2205_06973_amd.profiling issue <counters_a.csv> <counters_b.csv> <out.txt> "<command>"
    python -m paper_2205_06973_amd.profiling runs <kernel_trace.csv> <bench.json> <out.txt> "<command>" \
        [--kernel K] [--per-case N]
    python -m paper_2205_06973_amd.profiling kernel_traffic <fetch.csv> <write.csv> <stats.csv> <out.txt> \
        "<command>" --copy-bytes B --c64-bytes S64 --c128-bytes S128

`stats` condenses a `--kernel-trace --stats` kernel_stats.csv.  `traffic`
reads two `--pmc` counter_collection.csv files (FETCH_SIZE in one run,
WRITE_SIZE in the other; both in KiB per dispatch), scales each by what the
same counter reads for the plain copy kernel of known size (B bytes read and
B bytes written), and records the HBM bytes per part-pass launch, keyed by
workload and tagged with the kernel hash that bench.py printed for the
profiled run (roofline.kernel_hash: the generated part kernels).
`mfma` reads a `--pmc SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64
SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE` run and the matching kernel-trace
stats: per matrix-core kernel, flops per dispatch (MOPS x 512), achieved
TFLOP/s over the traced average duration, and the busy fraction of the SIMDs'
matrix cores (GRBM_GUI_ACTIVE is summed over the 8 XCDs; 1024 SIMDs).
`valu`, `waits` and `issue` summarise vector-ALU, wait-state and issue
counters the same way; `runs` splits a kernel trace into per-size runs of a
probe; `kernel_traffic` gives calibrated bytes per dispatch for every sweep
kernel of a run.
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "layout.h", "compile.cpp", "specialize.cpp"):
        with open(os.path.join(ROOT, "paper_2205_06973_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    base = name.split("(")[0]
    if "part_pass_spec" in base:  # one kernel per part (part_pass_spec_<i>): one row
        return "part_pass_spec"
    for tag in ("part_pass_kernel", "fused_pass_kernel", "gate_pass_1q",
                "gate_pass_2q", "set_basis_kernel", "norm_partial", "norm_final", "readout_kernel",
                "gather_kernel", "copy_probe_kernel"):
        if tag in base:
            tmpl = base[base.find(tag) + len(tag):]
            return tag + tmpl[:24]
    return base[:60]


def stats(csv_path: str, out_path: str, command: str, khash: str | None = None) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {command}",
             f"# kernel source hash: {kernel_source_hash()}"]
    if khash:
        lines.append(f"# kernel hash (generated part kernels): {khash}")
    lines += ["",
             f"{'kernel':48s} {'calls':>7s} {'avg_us':>11s} {'min_us':>11s} {'max_us':>11s} {'total_ms':>11s} {'pct':>6s}"]
    # rows with the same short name (the per-part specialized kernels) merge
    agg: dict[str, list[float]] = {}
    for r in rows:
        a = agg.setdefault(_short(r["Name"]), [0, 0.0, float("inf"), 0.0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
        a[2] = min(a[2], float(r["MinNs"]))
        a[3] = max(a[3], float(r["MaxNs"]))
        a[4] += float(r["Percentage"])
    for k, (calls, tot, mn, mx, pct) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{k:48s} {calls:7d} {tot / calls / 1e3:11.2f} {mn / 1e3:11.2f} {mx / 1e3:11.2f} "
                     f"{tot / 1e6:11.2f} {pct:6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _avg_ns(stats_csv: str) -> dict[str, float]:
    """Average duration per short kernel name (call-weighted over the rows a
    short name merges, such as the per-part specialized kernels)."""
    tot: dict[str, list[float]] = {}
    for r in csv.DictReader(open(stats_csv)):
        t = tot.setdefault(_short(r["Name"]), [0.0, 0])
        t[0] += float(r["TotalDurationNs"])
        t[1] += int(r["Calls"])
    return {k: v[0] / v[1] for k, v in tot.items() if v[1]}


def _counter_per_kernel(path: str, counter: str) -> dict[str, list[float]]:
    out: dict[str, list[float]] = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv: str, write_csv: str, key: str, command: str, copy_bytes: int,
            khash: str, txt_out: str | None = None, kernel: str = "part_pass_spec") -> dict:
    fetch = _counter_per_kernel(fetch_csv, "FETCH_SIZE")
    write = _counter_per_kernel(write_csv, "WRITE_SIZE")
    cf = [v for k, v in fetch.items() if k.startswith("copy_probe_kernel")][0]
    cw = [v for k, v in write.items() if k.startswith("copy_probe_kernel")][0]
    f_scale = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    w_scale = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    # only the profiled kernel (other part kernels in the same run, such as
    # the interpreter, are not part of the record)
    pf = [v for k, vs in fetch.items() if k == kernel for v in vs]
    pw = [v for k, vs in write.items() if k == kernel for v in vs]
    fb = sum(pf) / len(pf) * 1024.0 * f_scale
    wb = sum(pw) / len(pw) * 1024.0 * w_scale
    rec = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "launches_counted": len(pf), "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
           "command": command, "kernel_hash": khash}
    n, dt = key.split("_")[0][1:], key.split("_")[1]
    algo = 2 * (1 << int(n)) * (8 if dt == "c64" else 16)
    kib_f, kib_w = sum(pf) / len(pf), sum(pw) / len(pw)
    txt = [f"# HBM traffic per launch of {kernel}, workload {key}",
           f"# commands (run from /tmp with TMPDIR=/tmp, one counter per run): {command}",
           f"# kernel hash (generated part kernels): {khash}", "",
           f"calibration (copy_probe_kernel, {copy_bytes} B read + {copy_bytes} B written):",
           f"  FETCH_SIZE {sum(cf) / len(cf):14.1f} KiB -> scale {f_scale:.4f}",
           f"  WRITE_SIZE {sum(cw) / len(cw):14.1f} KiB -> scale {w_scale:.4f}", "",
           f"{kernel}, mean over {len(pf)} launches:",
           f"  FETCH_SIZE {kib_f:14.1f} KiB x {f_scale:.4f} = {fb / 1e9:.3f} GB",
           f"  WRITE_SIZE {kib_w:14.1f} KiB x {w_scale:.4f} = {wb / 1e9:.3f} GB",
           f"  total {(fb + wb) / 1e9:.3f} GB per launch; algorithmic 2 * 2^{n} * "
           f"{8 if dt == 'c64' else 16} B = {algo / 1e9:.3f} GB (ratio {(fb + wb) / algo:.5f})"]
    if txt_out:
        with open(txt_out, "w") as f:
            f.write("\n".join(txt) + "\n")
    print("\n".join(txt))
    path = os.path.join(PROFILES, "part_pass_traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d = {"workloads": d.get("workloads", {})}
    d["workloads"][key] = rec
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(rec, indent=1))
    return rec


def kernel_traffic(fetch_csv: str, write_csv: str, stats_csv: str, out_path: str, command: str,
                   copy_bytes: int, state_bytes: dict[str, int]) -> None:
    """Per kernel of a run: mean calibrated FETCH_SIZE + WRITE_SIZE bytes per
    dispatch against the algorithmic bytes of one sweep of its state (read
    + write every amplitude), with the traced average duration and the
    achieved fraction of the 8 TB/s HBM peak.  state_bytes maps a dtype tag
    ("float" / "double") to the state's bytes."""
    fetch = _counter_per_kernel(fetch_csv, "FETCH_SIZE")
    write = _counter_per_kernel(write_csv, "WRITE_SIZE")
    cf = [v for k, v in fetch.items() if k.startswith("copy_probe_kernel")][0]
    cw = [v for k, v in write.items() if k.startswith("copy_probe_kernel")][0]
    f_scale = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    w_scale = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    avg_ns = _avg_ns(stats_csv)
    lines = ["# HBM traffic and duration per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE;",
             "# durations from --kernel-trace --stats of the same command)",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             f"# calibration on copy_probe_kernel ({copy_bytes} B each way): FETCH x {f_scale:.4f}, "
             f"WRITE x {w_scale:.4f}", "",
             f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'GB/call':>9s} {'algo_GB':>9s} {'ratio':>6s} "
             f"{'GB/s':>8s} {'frac':>6s}"]
    for k in sorted(fetch):
        # kernels whose name carries the precision (the per-part specialized
        # kernels do not, and readouts are not sweeps)
        if k not in write or k not in avg_ns or not k.startswith(("fused_pass_kernel", "part_pass_kernel",
                                                                   "gate_pass")):
            continue
        tag = "double" if "double" in k else "float"
        if tag not in state_bytes:
            continue
        b = (sum(fetch[k]) / len(fetch[k]) * f_scale + sum(write[k]) / len(write[k]) * w_scale) * 1024.0
        algo = 2 * state_bytes[tag]
        gbs = algo / avg_ns[k]
        lines.append(f"{k:40s} {len(fetch[k]):6d} {avg_ns[k] / 1e3:10.1f} {b / 1e9:9.2f} {algo / 1e9:9.2f} "
                     f"{b / algo:6.3f} {gbs:8.1f} {gbs / 8000:6.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def mfma(counters_csv: str, stats_csv: str, out_path: str, command: str) -> None:
    ctr: dict[str, dict[str, list[float]]] = {}
    for r in csv.DictReader(open(counters_csv)):
        ctr.setdefault(_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    avg_ns = _avg_ns(stats_csv)
    peak = {"F32": 157.3, "F64": 78.6}
    lines = ["# matrix-core counters per dispatch (rocprofv3 --pmc) and kernel-trace durations",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             "# flops = MOPS * 512; util = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs * 1024 SIMDs)",
             "",
             f"{'kernel':36s} {'calls':>6s} {'avg_us':>10s} {'GFLOP/call':>11s} {'TFLOP/s':>8s} "
             f"{'peak':>6s} {'frac':>6s} {'busy_util':>9s}"]
    for k, d in sorted(ctr.items()):
        f32 = d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", [0.0])
        f64 = d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [0.0])
        kind = "F64" if sum(f64) > sum(f32) else "F32"
        mops = f64 if kind == "F64" else f32
        if sum(mops) == 0 or k not in avg_ns:
            continue
        flops = sum(mops) / len(mops) * 512
        busy = sum(d["SQ_VALU_MFMA_BUSY_CYCLES"]) / len(d["SQ_VALU_MFMA_BUSY_CYCLES"])
        gui = sum(d["GRBM_GUI_ACTIVE"]) / len(d["GRBM_GUI_ACTIVE"]) / 8
        tf = flops / avg_ns[k] / 1e3
        lines.append(f"{k:36s} {len(mops):6d} {avg_ns[k] / 1e3:10.1f} {flops / 1e9:11.1f} {tf:8.2f} "
                     f"{peak[kind]:6.1f} {tf / peak[kind]:6.3f} {busy / (gui * 1024):9.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_ACTIVE_INST_VALU",
                 "SQ_WAVES", "GRBM_GUI_ACTIVE")


def valu(counters_csv: str, stats_csv: str, out_path: str, command: str) -> None:
    """Vector-ALU summary of the part kernels: instructions per wavefront,
    the share that is the gates' own FMA/MUL arithmetic, and how busy the
    VALUs were (SQ_ACTIVE_INST_VALU counts 4-cycle issue slots per SIMD;
    GRBM_GUI_ACTIVE is summed over the 8 XCDs; 1024 SIMDs)."""
    ctr: dict[str, dict[str, list[float]]] = {}
    for r in csv.DictReader(open(counters_csv)):
        ctr.setdefault(_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    avg_ns = _avg_ns(stats_csv)
    lines = ["# vector-ALU counters per dispatch (rocprofv3 --pmc) and kernel-trace durations",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             "# arith = FMA + MUL instructions (F32 or F64) / all VALU instructions;",
             "# busy = SQ_ACTIVE_INST_VALU * 4 / (GRBM_GUI_ACTIVE / 8 * 1024 SIMDs)", "",
             f"{'kernel':36s} {'calls':>6s} {'avg_us':>10s} {'VALU/wave':>10s} {'arith':>6s} {'busy':>6s}"]
    mean = lambda d, c: sum(d.get(c, [0.0])) / max(1, len(d.get(c, [0.0])))  # noqa: E731
    for k, d in sorted(ctr.items()):
        if not k.startswith("part_pass") or "SQ_INSTS_VALU" not in d:
            continue
        v = mean(d, "SQ_INSTS_VALU")
        ar = sum(mean(d, c) for c in VALU_COUNTERS[1:5])
        waves = mean(d, "SQ_WAVES")
        busy = mean(d, "SQ_ACTIVE_INST_VALU") * 4 / (mean(d, "GRBM_GUI_ACTIVE") / 8 * 1024)
        lines.append(f"{k:36s} {len(d['SQ_INSTS_VALU']):6d} {avg_ns.get(k, 0) / 1e3:10.1f} "
                     f"{v / max(1.0, waves):10.0f} {ar / max(1.0, v):6.3f} {busy:6.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


WAIT_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS",
                 "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE")


def waits(counters_csv: str, stats_csv: str, out_path: str, command: str) -> None:
    """Where the part kernels' waves wait: per dispatch, the wave-cycles
    spent waiting on anything (SQ_WAIT_ANY), waiting to issue any
    instruction (SQ_WAIT_INST_ANY) and waiting to issue an LDS instruction
    (SQ_WAIT_INST_LDS), as shares of all wave-cycles (SQ_WAVE_CYCLES); plus
    how busy the LDS and VALU issue were (SQ_ACTIVE_INST_* count 4-cycle
    issue slots per SIMD; GRBM_GUI_ACTIVE is summed over the 8 XCDs; 1024
    SIMDs)."""
    ctr: dict[str, dict[str, list[float]]] = {}
    for r in csv.DictReader(open(counters_csv)):
        ctr.setdefault(_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    avg_ns = _avg_ns(stats_csv)
    mean = lambda d, c: sum(d.get(c, [0.0])) / max(1, len(d.get(c, [0.0])))  # noqa: E731
    lines = ["# wait-state counters per dispatch (rocprofv3 --pmc) and kernel-trace durations",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             "# wait_any, wait_issue, wait_lds = SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_WAIT_INST_LDS",
             "#   / SQ_WAVE_CYCLES; lds_of_waits = SQ_WAIT_INST_LDS / SQ_WAIT_ANY;",
             "# lds_busy, valu_busy = SQ_ACTIVE_INST_LDS, SQ_ACTIVE_INST_VALU * 4 / (GRBM_GUI_ACTIVE / 8 * 1024)",
             "",
             f"{'kernel':36s} {'calls':>6s} {'avg_us':>10s} {'wait_any':>9s} {'wait_issue':>10s} "
             f"{'wait_lds':>9s} {'lds_of_waits':>12s} {'lds_busy':>9s} {'valu_busy':>9s}"]
    for k, d in sorted(ctr.items()):
        if "SQ_WAVE_CYCLES" not in d or mean(d, "SQ_WAVE_CYCLES") == 0:
            continue
        cyc = mean(d, "SQ_WAVE_CYCLES")
        simd = mean(d, "GRBM_GUI_ACTIVE") / 8 * 1024
        lines.append(
            f"{k:36s} {len(d['SQ_WAVE_CYCLES']):6d} {avg_ns.get(k, 0) / 1e3:10.1f} "
            f"{mean(d, 'SQ_WAIT_ANY') / cyc:9.3f} {mean(d, 'SQ_WAIT_INST_ANY') / cyc:10.3f} "
            f"{mean(d, 'SQ_WAIT_INST_LDS') / cyc:9.4f} "
            f"{mean(d, 'SQ_WAIT_INST_LDS') / max(1.0, mean(d, 'SQ_WAIT_ANY')):12.4f} "
            f"{mean(d, 'SQ_ACTIVE_INST_LDS') * 4 / max(1.0, simd):9.3f} "
            f"{mean(d, 'SQ_ACTIVE_INST_VALU') * 4 / max(1.0, simd):9.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def issue(counters_a: str, counters_b: str, out_path: str, command: str) -> None:
    """Where the fused and part kernels' issue slots go: from one --pmc run,
    the share of wave cycles spent waiting on anything and waiting to issue,
    and how busy the VALU, scalar unit and matrix cores were; from a second,
    the instructions per wave by kind."""
    def load(path):
        d: dict[str, dict[str, list[float]]] = {}
        for r in csv.DictReader(open(path)):
            d.setdefault(_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        return d
    a, b = load(counters_a), load(counters_b)
    mean = lambda d, c: sum(d[c]) / len(d[c])  # noqa: E731
    lines = ["# issue counters per dispatch (two rocprofv3 --pmc runs of one command)",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             "# wait_any, wait_issue = SQ_WAIT_ANY, SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; valu, salu busy =",
             "# SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_SCA * 4 / (GRBM_GUI_ACTIVE / 8 * 1024 SIMDs); mfma busy =",
             "# SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 * 1024); per-wave counts from SQ_INSTS_*", "",
             f"{'kernel':36s} {'calls':>5s} {'wait_any':>8s} {'wait_iss':>8s} {'valu':>6s} {'salu':>6s} {'mfma':>6s}"
             f" {'VALU/w':>8s} {'SALU/w':>8s} {'MFMA/w':>8s} {'VMEMrd/w':>8s} {'VMEMwr/w':>8s}"]
    for k in sorted(a):
        if not k.startswith(("fused_pass_kernel", "part_pass")) or "SQ_WAVE_CYCLES" not in a[k]:
            continue
        d = a[k]
        wc = mean(d, "SQ_WAVE_CYCLES")
        simd = mean(d, "GRBM_GUI_ACTIVE") / 8 * 1024
        row = (f"{k:36s} {len(d['SQ_WAVES']):5d} {mean(d, 'SQ_WAIT_ANY') / wc:8.3f} {mean(d, 'SQ_WAIT_INST_ANY') / wc:8.3f}"
               f" {mean(d, 'SQ_ACTIVE_INST_VALU') * 4 / simd:6.3f} {mean(d, 'SQ_ACTIVE_INST_SCA') * 4 / simd:6.3f}"
               f" {mean(d, 'SQ_VALU_MFMA_BUSY_CYCLES') / simd:6.3f}")
        e = b.get(k)
        if e and "SQ_WAVES" in e:
            w = mean(e, "SQ_WAVES")
            row += (f" {mean(e, 'SQ_INSTS_VALU') / w:8.0f} {mean(e, 'SQ_INSTS_SALU') / w:8.0f}"
                    f" {mean(e, 'SQ_INSTS_VALU_MFMA_F32') / w:8.0f} {mean(e, 'SQ_INSTS_VMEM_RD') / w:8.0f}"
                    f" {mean(e, 'SQ_INSTS_VMEM_WR') / w:8.0f}")
        lines.append(row)
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def runs(trace_csv: str, bench_json: str, out_path: str, command: str, kernel: str = "gate_pass_1q",
         per_case: int = 16) -> None:
    """Per-case durations of a kernel from a --kernel-trace run of
    `bench.py --streaming-only`: its dispatches, in order, split into runs of
    `per_case` (the sweeps of one state size), matched with the bench's
    streaming rows (n, dtype) and their algorithmic bytes per sweep."""
    rows = [r for r in csv.DictReader(open(trace_csv)) if _short(r["Kernel_Name"]).startswith(kernel)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    with open(bench_json) as f:
        cases = json.loads(f.read().strip().splitlines()[-1])["streaming"]
    what = ("one sweep = H on qubit 0 (8 warm + 8 timed per size)" if kernel == "gate_pass_1q" else
            "one part, H twice on qubits 6-12, tile = qubits 0-12 (1 warm + 8 timed per size)")
    lines = [f"# per-size durations of {kernel} (rocprofv3 --kernel-trace), {what}",
             f"# command: {command}", f"# kernel source hash: {kernel_source_hash()}",
             f"# {len(dur)} dispatches in {per_case}-dispatch runs", "",
             f"{'n':>3s} {'dtype':>6s} {'avg_us':>10s} {'GB/s':>9s} {'frac':>6s} {'bench_GB/s':>11s}"]
    for i, c in enumerate(cases):
        run = dur[i * per_case:(i + 1) * per_case]
        if not run:
            break
        avg = sum(run) / len(run)
        b = 2 * (1 << c["n"]) * (8 if c["dtype"] == "c64" else 16)
        lines.append(f"{c['n']:3d} {c['dtype']:>6s} {avg:10.1f} {b / avg / 1e3:9.1f} {b / avg / 1e3 / 8000:6.3f} "
                     f"{c['pass_GBps']:11.1f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv):
    if argv[0] == "stats":
        stats(argv[1], argv[2], argv[3],
              argv[argv.index("--kernel-hash") + 1] if "--kernel-hash" in argv else None)
    elif argv[0] == "mfma":
        mfma(argv[1], argv[2], argv[3], argv[4])
    elif argv[0] == "valu":
        valu(argv[1], argv[2], argv[3], argv[4])
    elif argv[0] == "issue":
        issue(argv[1], argv[2], argv[3], argv[4])
    elif argv[0] == "waits":
        waits(argv[1], argv[2], argv[3], argv[4])
    elif argv[0] == "runs":
        kern = argv[argv.index("--kernel") + 1] if "--kernel" in argv else "gate_pass_1q"
        per = int(argv[argv.index("--per-case") + 1]) if "--per-case" in argv else 16
        runs(argv[1], argv[2], argv[3], argv[4], kern, per)
    elif argv[0] == "kernel_traffic":
        sb = {"float": int(argv[argv.index("--c64-bytes") + 1]),
              "double": int(argv[argv.index("--c128-bytes") + 1])}
        kernel_traffic(argv[1], argv[2], argv[3], argv[4], argv[5],
                       int(argv[argv.index("--copy-bytes") + 1]), sb)
    elif argv[0] == "traffic":
        cb = int(argv[argv.index("--copy-bytes") + 1])
        txt = argv[argv.index("--txt") + 1] if "--txt" in argv else None
        traffic(argv[1], argv[2], argv[3], argv[4], cb, argv[argv.index("--kernel-hash") + 1], txt)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
