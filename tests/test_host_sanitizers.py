"""The library's partitioners (Sec. IV) under AddressSanitizer + UBSan and
under ThreadSanitizer.

tests/host_san/partition_runner.cpp links the partitioning sources
(partition.cpp, dagp.cpp, gates.cpp) built with g++ and the sanitizer, runs
every strategy on a few circuits and limits (with and without the padding
qubits of a multi-level tile), and checks each partition exactly.  The part
counts must equal what libhisv.so returns for the same calls, and the
closure beam search, which runs on four helper threads in the runner, must
show no data race.
"""

import os
import shutil
import subprocess

import pytest

from paper_2205_06973_amd import hisv
from paper_2205_06973_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_06973_amd", "csrc")
RUNNER = os.path.join(ROOT, "tests", "host_san", "partition_runner.cpp")
GXX = shutil.which("g++")
pytestmark = pytest.mark.skipif(GXX is None, reason="needs g++")


def _build(workdir, sanitize):
    flags = ["-std=c++20", "-O1", "-g", f"-fsanitize={sanitize}", "-D__HIP_PLATFORM_AMD__",
             "-I/opt/rocm/include", "-I", CSRC]
    if sanitize != "thread":
        flags.append("-fno-sanitize-recover=all")
    exe = os.path.join(workdir, f"runner_{sanitize.replace(',', '_')}")
    srcs = [RUNNER] + [os.path.join(CSRC, f) for f in ("partition.cpp", "dagp.cpp", "gates.cpp")]
    r = subprocess.run([GXX] + flags + srcs + ["-o", exe, "-pthread"], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def runners(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("host_san"))
    return {"asan": _build(d, "address,undefined"), "tsan": _build(d, "thread")}


CIRCUITS = {
    "layered10": lambda: wl.layered28(1, n=10, layers=8),
    "random12": lambda: wl.random34(2, n=12, num_gates=300),
    "qft9": lambda: (9, wl.qft_circuit(9)),
    "random34": lambda: wl.random34(0, n=34, num_gates=1000),
}


def _jobs(name, n):
    if name == "random34":  # the headline circuit: the beam only
        return [("closure", 7, 0, 16, 0), ("closure", 5, 0, 8, 0), ("closure", 14, 0, 16, 6)]
    jobs = []
    for k in (2, 3, 5, 7):
        if k > n:
            continue
        jobs += [("nat", k, 0, 1, 0), ("dfs", k, 3, 4, 0), ("dagp", k, 3, 1, 0),
                 ("greedy", k, 3, 4, 0), ("closure", k, 0, 1, 0), ("closure", k, 0, 16, 0)]
    jobs += [("closure", 6, 0, 16, 2), ("greedy", 6, 3, 4, 2), ("dfs", 6, 3, 4, 2)]
    return jobs


def _files(tmp_path, name):
    n, gates = CIRCUITS[name]()
    c = tmp_path / f"{name}.txt"
    j = tmp_path / f"{name}_jobs.txt"
    with open(c, "w") as f:
        f.write(f"{n} {len(gates)}\n")
        for g in gates:
            f.write(f"{hisv.KINDS[g[0]]} {g[1]} {g[2]}\n")
    jobs = _jobs(name, n)
    with open(j, "w") as f:
        for job in jobs:
            f.write(" ".join(str(v) for v in job) + "\n")
    return n, gates, str(c), str(j), jobs


def _run(exe, c, j, env=None):
    r = subprocess.run([exe, c, j], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, **(env or {})))
    assert r.returncode == 0, r.stderr[-3000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-3000:]
    return [line.split(maxsplit=6) for line in r.stdout.splitlines()]


def _library_parts(n, gates, job):
    strategy, k, seed, trials, padq = job
    c = hisv.Circuit(n, gates)
    if padq:
        return hisv.Plan.partition_multilevel(c, k, padq, strategy, seed=seed, trials=trials).num_parts
    return hisv.Plan.partition(c, k, strategy, seed=seed, trials=trials).num_parts


@pytest.mark.parametrize("name", sorted(CIRCUITS))
def test_partitioners_under_asan_ubsan(runners, tmp_path, name):
    n, gates, c, j, jobs = _files(tmp_path, name)
    rows = _run(runners["asan"], c, j)
    assert len(rows) == len(jobs)
    for job, row in zip(jobs, rows):
        assert row[6] == "ok", (job, row)
        assert int(row[5]) == _library_parts(n, gates, job), (job, row)


@pytest.mark.parametrize("name", ["layered10", "random34"])
def test_closure_beam_threads_under_tsan(runners, tmp_path, name):
    _, _, c, j, jobs = _files(tmp_path, name)
    tsan = _run(runners["tsan"], c, j, {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    asan = _run(runners["asan"], c, j)
    assert [r[5] for r in tsan] == [r[5] for r in asan]
    assert all(r[6] == "ok" for r in tsan)
