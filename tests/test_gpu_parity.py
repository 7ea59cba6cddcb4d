"""GPU parity: the HIP path (through the C ABI) against the oracle.

Bars (max |delta amplitude| against the FP64 oracle, for circuits of at
most 10^4 gates): 1e-12 for complex128 states, 2e-5 for complex64 states,
plus an L2 bar of 1e-4 (complex64) / 1e-11 (complex128) on the whole
difference vector, because the max bar alone is loose once amplitudes are
themselves ~2^(-n/2).
"""

import math
import sys

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2205_06973_amd import hisv
from paper_2205_06973_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"c64": (2e-5, 1e-4), "c128": (1e-12, 1e-11)}
TDT = {"c64": torch.complex64, "c128": torch.complex128}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def new_state(n, dtype, init=0):
    t = torch.empty(1 << n, dtype=TDT[dtype], device="cuda")
    st = hisv.State.wrap_tensor(t, torch.cuda.current_stream())
    st.set_basis(init)
    return st


def run_hip(n, gates, dtype, k, strategy="dfs", mode="part_lds", init=0, seed=0, trials=16):
    print(f"[case] n={n} G={len(gates)} {dtype} k={k} {strategy} {mode}", flush=True)
    c = hisv.Circuit(n, gates)
    plan = hisv.Plan.partition(c, k, strategy, seed=seed, trials=trials)
    st = new_state(n, dtype, init)
    if mode == "gate_per_pass":
        st.simulate_gate_per_pass(c)
    elif mode == "auto_spec":  # AUTO over specialized gate-by-gate kernels
        plan.specialize(dtype)
        st.simulate(plan, "auto")
    else:
        st.simulate(plan, mode)
    out = st.amplitudes()
    st.close()
    return out, plan


def check(got, want, dtype):
    d = np.abs(got - want)
    mx, l2 = float(d.max()), float(np.linalg.norm(got - want))
    bar_max, bar_l2 = TOL[dtype]
    assert mx <= bar_max, f"max|d| = {mx:.3e} > {bar_max:.0e}"
    assert l2 <= bar_l2, f"||d||_2 = {l2:.3e} > {bar_l2:.0e}"
    return mx, l2


ALL = sv.ONE_QUBIT + sv.TWO_QUBIT


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["part_lds", "part_spec", "gate_per_pass"])
def test_random12_k4(dtype, mode):
    """The small workload: 12 qubits, 200 gates of {H, X, RZ, CX}, k = 4."""
    n, gates = wl.random12(0)
    got, plan = run_hip(n, gates, dtype, 4, "dfs", mode)
    check(got, sv.simulate(n, gates), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,k,strategy", [
    (1, 1, "nat"), (2, 2, "nat"), (3, 3, "dfs"), (5, 2, "dfs"), (6, 6, "nat"), (7, 3, "dfs"),
    (9, 5, "dfs"), (10, 7, "dfs"), (12, 12, "nat"), (13, 6, "dfs"), (14, 8, "dfs"),
    (16, 4, "nat"), (17, 7, "dfs"), (11, 6, "greedy"), (15, 7, "greedy"),
    (12, 5, "closure"), (16, 7, "closure"),
])
@pytest.mark.parametrize("mode", ["part_lds", "part_spec"])
def test_random_all_kinds(n, k, strategy, dtype, mode):
    kinds = ALL if n >= 2 else sv.ONE_QUBIT
    gates = wl.random_circuit(n, 150, kinds, seed=100 + n + k)
    if k > hisv.hs_max_part_qubits(dtype) and k < n:
        pytest.skip("part wider than the kernel tile for this dtype")
    got, _ = run_hip(n, gates, dtype, k, strategy, mode, init=(n * 7919) % (1 << n))
    check(got, sv.simulate(n, gates, (n * 7919) % (1 << n)), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["part_lds", "part_spec"])
def test_layered_20_k6(dtype, mode):
    n, gates = wl.layered28(3, n=20, layers=8)
    got, _ = run_hip(n, gates, dtype, 6, "dfs", mode)
    check(got, sv.simulate(n, gates), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode,strategy", [("part_lds", "dfs"), ("part_spec", "dagp"),
                                           ("part_lds", "closure"), ("part_spec", "closure")])
def test_qft_closed_form_18(dtype, mode, strategy):
    n = 18
    x = wl.random_basis_index(n, 5)
    got, _ = run_hip(n, wl.qft_circuit(n), dtype, 7, strategy, mode, init=x)
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    check(got, want, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,k,mode", [(9, 4, "part_fused"), (12, 5, "part_fused"),
                                      (16, 3, "part_fused"), (17, 5, "part_fused"),
                                      (10, 6, "part_fused"), (15, 6, "part_fused"),
                                      (11, 7, "part_fused"), (16, 7, "part_fused"),
                                      (15, 5, "auto"), (18, 7, "auto"),
                                      (14, 4, "auto_spec"), (17, 6, "auto_spec")])
def test_fused_and_auto(n, k, mode, dtype):
    # n = w + 4 is the smallest state the fused kernel takes (one tile)
    gates = wl.random_circuit(n, 160, ALL, seed=300 + n + k)
    got, _ = run_hip(n, gates, dtype, k, "dfs", mode, init=(n * 131) % (1 << n))
    check(got, sv.simulate(n, gates, (n * 131) % (1 << n)), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_qft_closed_form(dtype):
    # k = 7 parts of a QFT are dense 128 x 128 unitaries
    n = 17
    x = wl.random_basis_index(n, 9)
    got, _ = run_hip(n, wl.qft_circuit(n), dtype, 7, "dagp", "part_fused", init=x)
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    check(got, want, dtype)


def test_fused_rejects_wide_part():
    n, gates = wl.random34(1, n=14, num_gates=100)
    with pytest.raises(hisv.HisvError) as e:
        run_hip(n, gates, "c64", 8, "dfs", "part_fused")
    assert e.value.code == "HS_E_UNSUPPORTED"


def test_empty_circuit_leaves_state():
    st = new_state(10, "c64", init=37)
    c = hisv.Circuit(10, [])
    plan = hisv.Plan.partition(c, 4, "dfs")
    assert plan.num_parts == 0
    st.simulate(plan, "part_lds")
    want = sv.basis_state(10, 37)
    np.testing.assert_array_equal(st.amplitudes(), want)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_readout_norm_probabilities(dtype):
    n, gates = wl.random34(4, n=15, num_gates=200)
    c = hisv.Circuit(n, gates)
    plan = hisv.Plan.partition(c, 6, "dfs")
    st = new_state(n, dtype)
    st.simulate(plan, "part_lds")
    want = sv.simulate(n, gates)
    amp = st.amplitudes()
    check(amp, want, dtype)
    # slices, probabilities and the FP64 norm
    np.testing.assert_array_equal(st.amplitudes(1000, 77), amp[1000:1077])
    # probabilities of every amplitude against the oracle's |psi|^2: with
    # |a - psi| <= e, | |a|^2 - |psi|^2 | <= 2 e |psi| + e^2
    e = TOL[dtype][0]
    p_want = sv.probabilities(want)
    p = st.probabilities()
    assert p.size == want.size
    bar = 2 * e * np.abs(want) + e * e
    assert np.all(np.abs(p - p_want) <= bar), float(np.max(np.abs(p - p_want) - bar))
    np.testing.assert_array_equal(st.probabilities(5, 300), p[5:305])
    nrm = st.norm()
    assert abs(nrm - 1.0) < (1e-12 if dtype == "c128" else 1e-5)
    assert st.norm() == nrm  # fixed-order reduction: identical on every call


def test_part_by_part_equals_prefix():
    """The state after the first j parts equals the oracle after those parts' gates."""
    n, gates = wl.random34(9, n=14, num_gates=160)
    c = hisv.Circuit(n, gates)
    plan = hisv.Plan.partition(c, 5, "dfs", seed=2, trials=8)
    parts = plan.part_of_gate()
    st = new_state(n, "c128")
    for j in range(plan.num_parts):
        st.simulate_part(plan, j, "part_lds")
        if j in (0, plan.num_parts // 2, plan.num_parts - 1):
            prefix = [g for g, p in zip(gates, parts) if p <= j]
            check(st.amplitudes(), sv.simulate(n, prefix), "c128")


def test_errors_through_the_abi():
    c = hisv.Circuit(8, [("h", 0, -1, ())])
    plan = hisv.Plan.partition(c, 2, "nat")
    st = new_state(9, "c64")
    with pytest.raises(hisv.HisvError) as e:
        st.simulate(plan, "part_lds")
    assert e.value.code == "HS_E_ARG"
    with pytest.raises(hisv.HisvError):
        st.amplitudes(500, 100)
    with pytest.raises(hisv.HisvError):
        st.set_basis(1 << 9)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,strategy", [(12, "dfs"), (14, "nat"), (17, "dagp"), (18, "dfs"),
                                        (16, "closure"), (18, "greedy")])
@pytest.mark.parametrize("mode", ["part_lds", "part_spec"])
def test_multilevel_parity(n, strategy, mode, dtype):
    """Multi-level plans: parts fill the widest tile (14 / 13 qubits with padding)."""
    gates = wl.random_circuit(n, 300, ALL, seed=700 + n)
    init = (n * 104729) % (1 << n)
    print(f"[case] multilevel n={n} {dtype} {strategy} {mode}", flush=True)
    plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), strategy=strategy, dtype=dtype,
                                          seed=2, trials=8)
    st = new_state(n, dtype, init)
    st.simulate(plan, mode)
    got = st.amplitudes()
    st.close()
    check(got, sv.simulate(n, gates, init), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_multilevel_qft_closed_form(dtype):
    n = 18
    x = wl.random_basis_index(n, 11)
    plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, wl.qft_circuit(n)), strategy="dagp",
                                          dtype=dtype)
    st = new_state(n, dtype, x)
    st.simulate(plan, "part_spec")
    got = st.amplitudes()
    st.close()
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    check(got, want, dtype)


@pytest.mark.parametrize("dtype,tile", [("c64", 14), ("c128", 13)])
@pytest.mark.parametrize("lds_kib", [64, 16])
@pytest.mark.parametrize("n,strategy", [(15, "dfs"), (18, "dagp"), (17, "closure")])
def test_split_relayout_parity(n, strategy, dtype, tile, lds_kib):
    """Widest tiles, with LDS re-layouts run in 2 (64 KiB limit) or 4 (16 KiB)
    rounds over a quarter or half of the tile."""
    gates = wl.random_circuit(n, 300, ALL, seed=900 + n + tile)
    init = (n * 7) % (1 << n)
    print(f"[case] split n={n} {dtype} tile={tile} lds={lds_kib}KiB {strategy}", flush=True)
    hisv.hs_tune("spec_lds_limit_kib", lds_kib)
    try:
        plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gates), tile, 6, strategy, seed=4,
                                              trials=8)
        st = new_state(n, dtype, init)
        st.simulate(plan, "part_spec")
        got = st.amplitudes()
        st.close()
    finally:
        hisv.hs_tune("spec_lds_limit_kib", 64)
    check(got, sv.simulate(n, gates, init), dtype)


# ---- three-qubit kinds (decomposed at load) ----------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode,k", [("part_lds", 5), ("part_spec", 7), ("part_fused", 5), ("auto_spec", 6)])
def test_toffoli_fredkin_circuits(mode, k, dtype):
    n = 14
    gates = wl.random_circuit(n, 120, ("h", "u3", "rz", "cx", "cp", "ccx", "cswap"), seed=61)
    init = 12345 % (1 << n)
    got, _ = run_hip(n, gates, dtype, k, "dfs", mode, init=init)
    check(got, sv.simulate(n, gates, init), dtype)


def _adder_index(nb, a, b, carry=0):
    x = carry << (2 * nb + 1)
    for i in range(nb):
        x |= ((a >> i) & 1) << (2 + 2 * i)
        x |= ((b >> i) & 1) << (1 + 2 * i)
    return x


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adder_superposition(dtype):
    """H on every a_i, then the adder: amplitude 2^(-nb/2) on |a, a + b> for
    every a, zero elsewhere."""
    nb, b = 6, 45
    n, adder = wl.adder_circuit(nb)
    gates = [("h", 2 + 2 * i, -1, ()) for i in range(nb)] + adder
    got, _ = run_hip(n, gates, dtype, 7, "dfs", "part_spec", init=_adder_index(nb, 0, b))
    want = np.zeros(1 << n, dtype=np.complex128)
    for a in range(1 << nb):
        s = a + b
        want[_adder_index(nb, a, s % (1 << nb), s >> nb)] = 2 ** (-nb / 2)
    check(got, want, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("fuse", [1, 0])
def test_dense_two_qubit_ops(dtype, fuse):
    """Dressed two-qubit gates: the interpreter's 4 x 4 ops (on by default)
    against the oracle, and the same plan compiled without them."""
    n = 15
    gates = wl.dressed_pairs_circuit(n, 80, seed=7)
    hisv.hs_tune("fuse2", fuse)
    try:
        got, plan = run_hip(n, gates, dtype, 6, "dfs", "part_lds", init=4321)
        kinds = {int(k) for i in range(plan.num_parts)
                 for k in plan.part_descriptors(i, dtype, "part_lds")[2][:, 0]}
    finally:
        hisv.hs_tune("fuse2", 1)
    assert (9 in kinds) == bool(fuse)
    check(got, sv.simulate(n, gates, 4321), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["part_fused", "auto_spec", "part_spec"])
def test_deep_dense_five_qubit_parts(dtype, mode):
    """Dressed two-qubit blocks from a five-qubit window that dwells 16
    blocks (about 80 gates per part, k = 5): the fused dense-unitary kernel,
    AUTO over specialized and fused kernels (AUTO sends the deep parts to
    the fused kernel) and the specialized kernels alone, against the
    oracle."""
    n = 16
    gates = wl.dressed_pairs_circuit(n, 200, seed=3, span=5, dwell=16)
    got, plan = run_hip(n, gates, dtype, 5, "greedy", mode, init=1234)
    if mode == "auto_spec":
        assert plan.auto_choice(dtype).sum() >= 1
    check(got, sv.simulate(n, gates, 1234), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode,shape", [("part_fused", 0), ("part_fused", 1), ("part_fused", 2),
                                        ("auto_spec", -1)])
def test_fused_persistent_grid_24_qubits(dtype, mode, shape):
    """Fused five-qubit parts on a 24-qubit state, where each workgroup of
    the software-pipelined fused kernel walks many tile groups: two
    dressed-pair circuits on qubits 0-11 and 12-23, interleaved, so the
    state is psi_low * psi_high and every amplitude is checked against the
    oracle's two 12-qubit states.  Parts on the high half run with coalesced
    columns, parts on qubits 0..3 without.  Every launch shape of the
    four- and five-qubit fused kernels."""
    n, nl = 24, 12
    gates, lo, hi = wl.split_dressed_circuit(n, nl, 120, seed=5)
    hisv.hs_tune("fused_shape", shape)  # the three launch shapes
    try:
        got, plan = run_hip(n, gates, dtype, 5, "greedy", mode)
    finally:
        hisv.hs_tune("fused_shape", -1)
    if mode == "auto_spec":
        assert plan.auto_choice(dtype).sum() >= 1
    want = np.kron(sv.simulate(n - nl, hi), sv.simulate(nl, lo))
    check(got, want, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_background_specialization(dtype):
    """hs_plan_specialize_async: AUTO runs the interpreter while the kernels
    build and the specialized kernels once they are there; both results
    match the oracle, and the plan reports the build."""
    n, gates = wl.random12(3)
    want = sv.simulate(n, gates)
    plan = hisv.Plan.partition(hisv.Circuit(n, gates), 4, "greedy", seed=0, trials=8)
    print(f"[case] background specialization {dtype}", flush=True)
    plan.specialize_async(dtype)
    st = new_state(n, dtype)
    st.simulate(plan, "auto")  # interpreter or specialized, whichever is ready
    check(st.amplitudes(), want, dtype)
    plan.specialize_wait(dtype)
    assert plan.specialized(dtype)
    st.set_basis(0)
    st.simulate(plan, "auto")
    check(st.amplitudes(), want, dtype)
    st.close()
