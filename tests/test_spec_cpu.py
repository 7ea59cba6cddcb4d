"""The generated specialized part kernels, run on the host.

Each part's kernel source (exactly what hipRTC compiles for gfx950) is built
with g++ against tests/spec_cpu/prelude.h, which maps the few HIP constructs
the generator emits onto std::thread and std::barrier, and run with
AddressSanitizer and UBSan.  The resulting state must match the oracle, and
no access may leave the state or the LDS array.  This covers on the CPU the
parts of the specialized path that descriptor replays do not: the emitted
LDS re-layouts (including split ones), the XCD-contiguous tile walk, the
persistent-grid loop and the 64-bit address arithmetic.
"""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import statevector as sv  # noqa: E402
from paper_2205_06973_amd import hisv  # noqa: E402
from paper_2205_06973_amd import workloads as wl  # noqa: E402

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spec_cpu")
GXX = shutil.which("g++")
pytestmark = pytest.mark.skipif(GXX is None, reason="needs g++")


def build_runner(plan, dtype, workdir):
    parts = []
    calls = []
    for i in range(plan.num_parts):
        src = plan.part_source(i, dtype).replace('extern "C" ', "")
        parts.append(f"namespace part{i} {{\n{src}\n}}  // namespace part{i}\n")
        calls.append(f"    case {i}: part{i}::part_pass_spec((part{i}::V*)st, tiles, xcd); break;\n")
    with open(os.path.join(workdir, "parts.inc"), "w") as f:
        f.write("".join(parts))
        f.write("inline void launch_part(int part, unsigned char* st, unsigned long long tiles, "
                "unsigned xcd) {\n  switch (part) {\n" + "".join(calls) + "    default: std::abort();\n  }\n}\n")
    exe = os.path.join(workdir, "runner")
    cmd = [GXX, "-std=c++20", "-O0", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIPCC_RTC__", "-I", HERE, "-I", workdir,
           os.path.join(HERE, "runner.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def launches(plan, n, dtype, persistent):
    """Grid shapes the library's launcher can produce: one workgroup per tile,
    or a persistent grid of a quarter of the tiles; XCD-contiguous runs when
    the grid and tile count allow."""
    lines = []
    for i in range(plan.num_parts):
        hdr, _, _ = plan.part_descriptors(i, dtype, "part_spec")
        m, wb = int(hdr[0]), int(hdr[2])
        tiles = 1 << (n - m)
        grid = max(1, tiles // 4) if persistent else tiles
        xcd = 0
        if tiles % 8 == 0 and grid >= 8:
            grid -= grid % 8
            xcd = 1
        lines.append(f"{i} {grid} {64 << wb} {tiles} {xcd}\n")
    return "".join(lines)


def run_on_host(plan, n, dtype, psi0, tmp_path, persistent=False):
    exe = build_runner(plan, dtype, str(tmp_path))
    cdt = np.complex64 if dtype == "c64" else np.complex128
    state = os.path.join(str(tmp_path), "state.bin")
    np.ascontiguousarray(psi0.astype(cdt)).tofile(state)
    lf = os.path.join(str(tmp_path), "launches.txt")
    with open(lf, "w") as f:
        f.write(launches(plan, n, dtype, persistent))
    r = subprocess.run([exe, state, lf], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return np.fromfile(state, dtype=cdt).astype(np.complex128)


def random_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


TOL = {"c64": 2e-5, "c128": 1e-12}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("persistent", [False, True])
def test_spec_kernels_k7(dtype, persistent, tmp_path):
    n = 16
    gates = wl.random_circuit(n, 90, sv.ONE_QUBIT + sv.TWO_QUBIT, seed=41)
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), 7, "dfs", seed=1, trials=16)
    psi0 = random_state(n, 5)
    got = run_on_host(plan, n, dtype, psi0, tmp_path, persistent)
    np.testing.assert_allclose(got, sv.simulate(n, gates, psi0), atol=TOL[dtype], rtol=0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_spec_kernels_multilevel_split(dtype, tmp_path):
    """Widest tiles: every LDS re-layout runs in two rounds over half the tile."""
    n = 17
    gates = wl.random_circuit(n, 120, sv.ONE_QUBIT + sv.TWO_QUBIT, seed=43)
    plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), strategy="dfs", dtype=dtype,
                                          seed=2, trials=8)
    src = plan.part_source(0, dtype)
    assert "lds[" in src
    psi0 = random_state(n, 6)
    got = run_on_host(plan, n, dtype, psi0, tmp_path)
    np.testing.assert_allclose(got, sv.simulate(n, gates, psi0), atol=TOL[dtype], rtol=0)


def test_spec_kernels_four_round_relayouts(tmp_path):
    """A 16 KiB LDS limit on 13-qubit tiles (64 KiB): re-layouts run in four
    rounds over a quarter of the tile."""
    n = 15
    gates = wl.random_circuit(n, 100, sv.ONE_QUBIT + sv.TWO_QUBIT, seed=44)
    hisv.hs_tune("spec_lds_limit_kib", 16)
    try:
        plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), 13, 6, "dagp", seed=3)
        # some part's LDS array is a quarter of its tile (four rounds)
        quarter = False
        for i in range(plan.num_parts):
            m = int(plan.part_descriptors(i, "c64", "part_spec")[0][0])
            quarter |= f"__shared__ V lds[{1 << (m - 2)}];" in plan.part_source(i, "c64")
        assert quarter
        psi0 = random_state(n, 7)
        got = run_on_host(plan, n, "c64", psi0, tmp_path)
    finally:
        hisv.hs_tune("spec_lds_limit_kib", 64)
    np.testing.assert_allclose(got, sv.simulate(n, gates, psi0), atol=TOL["c64"], rtol=0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_spec_kernels_with_dense_two_qubit_ops(dtype, tmp_path):
    """Two-qubit gates merged with the dense one-qubit gates around them into
    4 x 4 ops (off by default for these kernels, on here): the merge in the
    part compiler and the emitted 4 x 4 code, on layered U3 + CX circuits
    and on every two-qubit kind."""
    n = 14
    gates = wl.layered_circuit(n, 6, seed=45) + wl.random_circuit(
        n, 60, ("u3", "cx", "cz", "cp", "swap", "h", "rz"), seed=46)
    hisv.hs_tune("spec_fuse2", 1)
    try:
        plan = hisv.Plan.partition(hisv.Circuit(n, gates), 6, "dfs", seed=4, trials=8)
        kinds = {int(k) for i in range(plan.num_parts)
                 for k in plan.part_descriptors(i, dtype, "part_spec")[2][:, 0]}
        assert 9 in kinds  # some 4 x 4 ops were formed
        psi0 = random_state(n, 8)
        got = run_on_host(plan, n, dtype, psi0, tmp_path)
    finally:
        hisv.hs_tune("spec_fuse2", 0)
    np.testing.assert_allclose(got, sv.simulate(n, gates, psi0), atol=TOL[dtype], rtol=0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_spec_kernels_prefetch_with_split_relayouts(dtype, tmp_path):
    """Persistent grid with next-tile prefetch on the widest tiles, whose LDS
    re-layouts run in two rounds: the rounds must not land in the registers
    that hold the prefetched tile."""
    n = 17
    gates = wl.random_circuit(n, 120, sv.ONE_QUBIT + sv.TWO_QUBIT, seed=43)
    hisv.hs_tune("spec_grid", 1)
    hisv.hs_tune("spec_prefetch", 1)
    try:
        plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), strategy="dfs", dtype=dtype,
                                              seed=2, trials=8)
        srcs = [plan.part_source(i, dtype) for i in range(plan.num_parts)]
        # prefetch registers and split-round registers both present
        assert any(" nr0" in s and " sr0" in s for s in srcs)
        psi0 = random_state(n, 6)
        got = run_on_host(plan, n, dtype, psi0, tmp_path, persistent=True)
    finally:
        hisv.hs_tune("spec_grid", 0)
        hisv.hs_tune("spec_prefetch", 0)
    np.testing.assert_allclose(got, sv.simulate(n, gates, psi0), atol=TOL[dtype], rtol=0)
