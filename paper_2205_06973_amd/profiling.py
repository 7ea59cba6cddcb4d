"""Turn rocprofv3 output into the committed kernel summaries under profiles/.

    python -m paper_2205_06973_amd.profiling stats  <stats.csv> <out.txt> "<command>"
    python -m paper_2205_06973_amd.profiling traffic <fetch.csv> <write.csv> <key> "<command>" \
        --copy-bytes B

`stats` condenses a `--kernel-trace --stats` kernel_stats.csv.  `traffic`
reads two `--pmc` counter_collection.csv files (FETCH_SIZE in one run,
WRITE_SIZE in the other; both in KiB per dispatch), scales each by what the
same counter reads for the plain copy kernel of known size (B bytes read and
B bytes written), and records the HBM bytes per part-pass launch, keyed by
workload and tagged with the hash of the kernel sources it was taken on.
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
    for tag in ("part_pass_spec", "part_pass_kernel", "fused_pass_kernel", "gate_pass_1q",
                "gate_pass_2q", "set_basis_kernel", "norm_partial", "norm_final", "readout_kernel",
                "gather_kernel", "copy_probe_kernel"):
        if tag in base:
            tmpl = base[base.find(tag) + len(tag):]
            return tag + tmpl[:24]
    return base[:60]


def stats(csv_path: str, out_path: str, command: str) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {command}",
             f"# kernel source hash: {kernel_source_hash()}", "",
             f"{'kernel':48s} {'calls':>7s} {'avg_us':>11s} {'min_us':>11s} {'max_us':>11s} {'total_ms':>11s} {'pct':>6s}"]
    for r in rows:
        lines.append(f"{_short(r['Name']):48s} {int(r['Calls']):7d} {float(r['AverageNs'])/1e3:11.2f} "
                     f"{float(r['MinNs'])/1e3:11.2f} {float(r['MaxNs'])/1e3:11.2f} "
                     f"{float(r['TotalDurationNs'])/1e6:11.2f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_per_kernel(path: str, counter: str) -> dict[str, list[float]]:
    out: dict[str, list[float]] = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv: str, write_csv: str, key: str, command: str, copy_bytes: int) -> dict:
    fetch = _counter_per_kernel(fetch_csv, "FETCH_SIZE")
    write = _counter_per_kernel(write_csv, "WRITE_SIZE")
    cf = [v for k, v in fetch.items() if k.startswith("copy_probe_kernel")][0]
    cw = [v for k, v in write.items() if k.startswith("copy_probe_kernel")][0]
    f_scale = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    w_scale = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    pf = [v for k, vs in fetch.items() if k.startswith("part_pass") for v in vs]
    pw = [v for k, vs in write.items() if k.startswith("part_pass") for v in vs]
    fb = sum(pf) / len(pf) * 1024.0 * f_scale
    wb = sum(pw) / len(pw) * 1024.0 * w_scale
    rec = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "launches_counted": len(pf), "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
           "command": command}
    path = os.path.join(PROFILES, "part_pass_traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    if d.get("kernel_source_hash") != kernel_source_hash():
        d = {"kernel_source_hash": kernel_source_hash(), "workloads": {}}
    d["workloads"][key] = rec
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(rec, indent=1))
    return rec


def main(argv):
    if argv[0] == "stats":
        stats(argv[1], argv[2], argv[3])
    elif argv[0] == "traffic":
        cb = int(argv[argv.index("--copy-bytes") + 1])
        traffic(argv[1], argv[2], argv[3], argv[4], cb)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
