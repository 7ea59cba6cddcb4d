"""Host-side tests of the rocprofv3 summaries (paper_2205_06973_amd/profiling.py)
on synthetic CSV files with known values: the per-kernel merging of the
specialized kernels, call-weighted averages, the copy-probe calibration of
the traffic counters and the algorithmic-byte ratio."""

import csv
import json

from paper_2205_06973_amd import profiling

STATS_HEAD = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
CTR_HEAD = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, head, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(head)
        w.writerows(rows)
    return str(path)


def test_stats_merges_specialized_kernels_call_weighted(tmp_path):
    src = _write(tmp_path / "s.csv", STATS_HEAD, [
        ["part_pass_spec_0", 3, 300_000, 100_000, 30.0, 90_000, 110_000, 0],
        ["part_pass_spec_1", 1, 200_000, 200_000, 20.0, 200_000, 200_000, 0],
        ["void hisv::norm_final(double const*, double*)", 2, 10_000, 5_000, 1.0, 4_000, 6_000, 0],
    ])
    out = tmp_path / "s.txt"
    profiling.stats(src, str(out), "cmd", khash="abc")
    text = out.read_text()
    row = [l for l in text.splitlines() if l.startswith("part_pass_spec")][0].split()
    # 4 calls, 500 us in all: 125 us a call, min 90, max 200
    assert row[1:6] == ["4", "125.00", "90.00", "200.00", "0.50"]
    assert "kernel hash (generated part kernels): abc" in text
    avg = profiling._avg_ns(src)
    assert avg["part_pass_spec"] == 125_000 and avg["norm_final"] == 5_000


def test_traffic_calibrates_on_the_copy_probe(tmp_path, monkeypatch):
    monkeypatch.setattr(profiling, "PROFILES", str(tmp_path))
    copy_bytes = 1 << 30
    # the copy reads and writes copy_bytes: FETCH_SIZE reports half, WRITE_SIZE all of it (KiB)
    fetch = _write(tmp_path / "f.csv", CTR_HEAD, [
        ["copy_probe_kernel(...)", "FETCH_SIZE", copy_bytes / 2 / 1024],
        ["part_pass_spec_3", "FETCH_SIZE", (1 << 20) / 1024],
        ["part_pass_spec_4", "FETCH_SIZE", (1 << 20) / 1024],
    ])
    write = _write(tmp_path / "w.csv", CTR_HEAD, [
        ["copy_probe_kernel(...)", "WRITE_SIZE", copy_bytes / 1024],
        ["part_pass_spec_3", "WRITE_SIZE", (2 << 20) / 1024],
        ["part_pass_spec_4", "WRITE_SIZE", (2 << 20) / 1024],
    ])
    rec = profiling.traffic(fetch, write, "n20_c64_k7", "cmd", copy_bytes, "h1", str(tmp_path / "t.txt"))
    assert abs(rec["copy_fetch_scale"] - 2.0) < 1e-12 and abs(rec["copy_write_scale"] - 1.0) < 1e-12
    assert rec["fetch_bytes_per_launch"] == 2 << 20 and rec["write_bytes_per_launch"] == 2 << 20
    assert rec["launches_counted"] == 2
    # 2 * 2^20 * 8 B algorithmic = 16 MiB; counted 4 MiB: ratio 0.25
    assert "(ratio 0.25000)" in (tmp_path / "t.txt").read_text()
    saved = json.load(open(tmp_path / "part_pass_traffic.json"))
    assert saved["workloads"]["n20_c64_k7"]["kernel_hash"] == "h1"


def test_kernel_traffic_per_precision(tmp_path):
    copy_bytes = 1 << 30
    fetch = _write(tmp_path / "f.csv", CTR_HEAD, [
        ["copy_probe_kernel(...)", "FETCH_SIZE", copy_bytes / 2 / 1024],
        ["void hisv::fused_pass_kernel<float, 5, false>(...)", "FETCH_SIZE", (8 << 20) / 2 / 1024],
    ])
    write = _write(tmp_path / "w.csv", CTR_HEAD, [
        ["copy_probe_kernel(...)", "WRITE_SIZE", copy_bytes / 1024],
        ["void hisv::fused_pass_kernel<float, 5, false>(...)", "WRITE_SIZE", (8 << 20) / 1024],
    ])
    stats = _write(tmp_path / "s.csv", STATS_HEAD, [
        ["void hisv::fused_pass_kernel<float, 5, false>(...)", 2, 4_000, 2_000, 1.0, 2_000, 2_000, 0],
    ])
    out = tmp_path / "k.txt"
    profiling.kernel_traffic(fetch, write, stats, str(out), "cmd", copy_bytes, {"float": 8 << 20, "double": 16 << 20})
    row = [l for l in out.read_text().splitlines() if l.startswith("fused_pass_kernel")][0].split()
    # 16 MiB counted against 16 MiB algorithmic in 2 us: ratio 1, 8.39 TB/s
    assert row[-3] == "1.000" and abs(float(row[-2]) - (16 << 20) / 2_000) < 0.1
