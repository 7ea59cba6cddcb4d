"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (specialized part kernels).

The oracle cannot hold these states on the host (complex128 at 32-34 qubits
is 64-256 GiB), so each check uses outputs it can compute one by one or a
property that holds at any size:

* product-block circuits (two-qubit gates only inside the even or inside the
  odd qubits): the state is psi_even(even bits) * psi_odd(odd bits), each
  factor from the oracle at n/2 qubits -- compared at sampled indices;
* QFT of a basis state: every amplitude has a closed form;
* the real random / layered circuits: U followed by its inverse returns
  |0...0>, and the norm stays 1.
"""

import math

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2205_06973_amd import hisv
from paper_2205_06973_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"c64": 2e-5, "c128": 1e-12}
TDT = {"c64": torch.complex64, "c128": torch.complex128}


@pytest.fixture(autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def simulate(n, gates, dtype, k, strategy, mode="part_spec", init=0, extra=None):
    print(f"[case] n={n} G={len(gates)} {dtype} k={k} {strategy} {mode}", flush=True)
    buf = torch.empty(1 << n, dtype=TDT[dtype], device="cuda")
    st = hisv.State.wrap_tensor(buf, torch.cuda.current_stream())
    st.set_basis(init)
    trials = 16 if strategy.endswith("closure") else 32  # closure: the bench's draws
    for gs in [gates] + ([extra] if extra else []):
        if strategy.startswith("ml-"):  # multi-level: parts fill the kernel tile
            plan = hisv.Plan.partition_multilevel(hisv.Circuit(n, gs), strategy=strategy[3:],
                                                  dtype=dtype, seed=0, trials=trials)
        else:
            plan = hisv.Plan.partition(hisv.Circuit(n, gs), k, strategy, seed=0, trials=trials)
        if mode == "auto_spec":  # AUTO over specialized gate-by-gate and fused kernels
            plan.specialize(dtype)
            st.simulate(plan, "auto")
        else:
            st.simulate(plan, mode)
    st.sync()
    return st, buf


def product_factors(n, gates):
    ren = lambda g: (g[0], g[1] // 2, g[2] // 2 if g[2] >= 0 else -1, g[3])  # noqa: E731
    pe = sv.simulate((n + 1) // 2, [ren(g) for g in gates if g[1] % 2 == 0])
    po = sv.simulate(n // 2, [ren(g) for g in gates if g[1] % 2 == 1])
    return pe, po


def product_amp(idx, n, pe, po):
    ie = np.zeros_like(idx)
    io = np.zeros_like(idx)
    for b in range((n + 1) // 2):
        ie |= ((idx >> np.uint64(2 * b)) & np.uint64(1)) << np.uint64(b)
    for b in range(n // 2):
        io |= ((idx >> np.uint64(2 * b + 1)) & np.uint64(1)) << np.uint64(b)
    return pe[ie.astype(np.int64)] * po[io.astype(np.int64)]


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.concatenate([np.arange(4096, dtype=np.uint64), idx,
                           np.arange((1 << n) - 4096, 1 << n, dtype=np.uint64)])


def report(name, d, n):
    mx = float(np.max(d))
    print(f"[{name}] max|d| = {mx:.3e}, max|d|*2^(n/2) = {mx * 2 ** (n / 2):.3e}", flush=True)
    return mx


@pytest.mark.parametrize("n,dtype,k,strategy,layers", [
    (28, "c64", 6, "dfs", 40), (28, "c128", 6, "dfs", 40)])
def test_layered28_product_block(n, dtype, k, strategy, layers):
    gates = wl.layered_product_block_circuit(n, layers, seed=1)
    st, buf = simulate(n, gates, dtype, k, strategy)
    pe, po = product_factors(n, gates)
    idx = sample_indices(n, 1 << 20, 2)
    d = np.abs(st.amplitudes_at(idx) - product_amp(idx, n, pe, po))
    assert report("layered28 product", d, n) <= TOL[dtype]
    assert abs(st.norm() - 1) <= (1e-5 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_layered28_round_trip(dtype):
    n, gates = wl.layered28(0)
    st, buf = simulate(n, gates, dtype, 6, "dfs", extra=sv.inverse_circuit(gates))
    idx = sample_indices(n, 1 << 14, 3)
    got = st.amplitudes_at(idx)
    want = np.zeros(idx.size, dtype=np.complex128)
    want[idx == 0] = 1.0
    assert report("layered28 U^-1 U", np.abs(got - want), n) <= TOL[dtype]


@pytest.mark.parametrize("strategy,mode", [("dagp", "part_spec"), ("ml-dagp", "part_spec"),
                                           ("greedy", "part_spec"), ("ml-greedy", "part_spec"),
                                           ("closure", "part_spec"), ("ml-closure", "part_spec"),
                                           ("greedy", "part_fused"), ("closure", "auto_spec")])
def test_qft32_closed_form(strategy, mode):
    """The 32-qubit QFT on a random basis state (32 GiB complex64), k = 7:
    gate-by-gate specialized kernels, the fused dense-unitary kernels on
    matrix cores, and AUTO over both; 2^24 random amplitudes and the first
    and last 4,096 against the closed form."""
    n, gates, x = wl.qft32(0)
    st, buf = simulate(n, gates, "c64", 7, strategy, mode=mode, init=x)
    idx = sample_indices(n, 1 << 24, 4)
    want = np.exp(2j * np.pi * ((np.uint64(x) * idx) % np.uint64(1 << n)).astype(np.float64)
                  / (1 << n)) / math.sqrt(1 << n)
    d = np.abs(st.amplitudes_at(idx) - want)
    assert report("qft32", d, n) <= TOL["c64"]
    assert abs(st.norm() - 1) <= 1e-5


@pytest.mark.parametrize("n,dtype,strategy", [(34, "c64", "dfs"), (33, "c128", "dfs"),
                                              (34, "c64", "ml-dfs"), (33, "c128", "ml-dfs"),
                                              (34, "c64", "greedy"), (33, "c128", "ml-greedy"),
                                              (34, "c64", "closure"), (33, "c128", "closure"),
                                              (34, "c64", "ml-closure")])
def test_random34_product_block(n, dtype, strategy):
    gates = wl.product_block_circuit(n, 1000, wl.RANDOM34_KINDS, seed=5)
    st, buf = simulate(n, gates, dtype, 7, strategy)
    pe, po = product_factors(n, gates)
    idx = sample_indices(n, 1 << 20, 6)
    d = np.abs(st.amplitudes_at(idx) - product_amp(idx, n, pe, po))
    assert report(f"random{n} product", d, n) <= TOL[dtype]
    assert abs(st.norm() - 1) <= (1e-5 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("k,mode", [(5, "part_spec"), (6, "part_spec"), (7, "part_lds")])
def test_random34_product_block_k_and_interpreter(k, mode):
    """The 34-qubit complex64 workload's k sweep (5 and 6, specialized
    kernels) and the interpreter kernel at k = 7, on the product-block
    variant of its gate distribution."""
    n, dtype = 34, "c64"
    gates = wl.product_block_circuit(n, 1000, wl.RANDOM34_KINDS, seed=5)
    st, buf = simulate(n, gates, dtype, k, "closure", mode=mode)
    pe, po = product_factors(n, gates)
    idx = sample_indices(n, 1 << 20, 6 + k)
    d = np.abs(st.amplitudes_at(idx) - product_amp(idx, n, pe, po))
    assert report(f"random{n} product k={k} {mode}", d, n) <= TOL[dtype]
    assert abs(st.norm() - 1) <= 1e-5


@pytest.fixture(scope="module")
def headline22():
    """The headline gate distribution (1,000 gates over {H, RZ, RX, CX, CZ})
    at 22 qubits, and the oracle's full state for it."""
    n, gates = wl.random34(0, n=22)
    print("[case] oracle, random22 (1,000 gates)", flush=True)
    return n, gates, sv.simulate(n, gates)


@pytest.mark.parametrize("strategy", ["closure", "greedy"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_headline_configuration_full_vector(dtype, strategy, headline22):
    """The headline launch configuration -- closure partition (and the
    greedy one), k = 7, specialized kernels -- against the oracle on every
    amplitude at 22 qubits (max |d| and ||d||_2 bars)."""
    n, gates, want = headline22
    st, buf = simulate(n, gates, dtype, 7, strategy)
    got = st.amplitudes()
    d = np.abs(got - want)
    report(f"random{n} full vector {dtype}", d, n)
    bar_max, bar_l2 = {"c64": (2e-5, 1e-4), "c128": (1e-12, 1e-11)}[dtype]
    assert float(d.max()) <= bar_max
    assert float(np.linalg.norm(got - want)) <= bar_l2


@pytest.mark.parametrize("n,dtype", [(35, "c64"), (34, "c128")])
def test_largest_state_round_trip(n, dtype):
    """The largest power-of-two states that fit 288 GB of HBM (256 GiB)."""
    if torch.cuda.mem_get_info()[0] < (1 << n) * (8 if dtype == "c64" else 16) + (4 << 30):
        pytest.skip("device memory below the 256 GiB state plus 4 GiB headroom")
    _, gates = wl.random34(1, n=n, num_gates=200)
    st, buf = simulate(n, gates, dtype, 7, "dfs", extra=sv.inverse_circuit(gates))
    idx = sample_indices(n, 1 << 14, 8)
    got = st.amplitudes_at(idx)
    want = np.zeros(idx.size, dtype=np.complex128)
    want[idx == 0] = 1.0
    assert report(f"random{n} {dtype} U^-1 U", np.abs(got - want), n) <= TOL[dtype]
    assert abs(st.norm() - 1) <= (1e-5 if dtype == "c64" else 1e-12)
    st.close()
    del buf


@pytest.mark.parametrize("n,dtype", [(34, "c64"), (33, "c128")])
def test_random34_round_trip(n, dtype):
    _, gates = wl.random34(0, n=n)
    # the headline configuration: closure partition, k = 7, specialized kernels
    st, buf = simulate(n, gates, dtype, 7, "closure", extra=sv.inverse_circuit(gates))
    idx = sample_indices(n, 1 << 14, 7)
    got = st.amplitudes_at(idx)
    want = np.zeros(idx.size, dtype=np.complex128)
    want[idx == 0] = 1.0
    assert report(f"random{n} U^-1 U", np.abs(got - want), n) <= TOL[dtype]


def test_adder16_superposition_34_qubits():
    """A 16-bit ripple-carry adder (34 qubits, complex64, 545 gates after the
    Toffoli decompositions) on |a = uniform superposition over 2^16, b>:
    amplitude 2^-8 on |a, a + b> for every a; sampled exactly."""
    nb, b = 16, 40503
    n, adder = wl.adder_circuit(nb)
    gates = [("h", 2 + 2 * i, -1, ()) for i in range(nb)] + adder

    def index(a, bb, carry=0):
        x = np.uint64(carry) << np.uint64(2 * nb + 1)
        for i in range(nb):
            x |= np.uint64((a >> i) & 1) << np.uint64(2 + 2 * i)
            x |= np.uint64((bb >> i) & 1) << np.uint64(1 + 2 * i)
        return x

    st, buf = simulate(n, gates, "c64", 7, "dfs", init=int(index(0, b)))
    rng = np.random.default_rng(12)
    avals = rng.integers(0, 1 << nb, 2048)
    idx = np.array([index(int(a), (int(a) + b) % (1 << nb), (int(a) + b) >> nb) for a in avals],
                   dtype=np.uint64)
    got = st.amplitudes_at(idx)
    assert report("adder16 hits", np.abs(got - 2.0 ** -8), n) <= TOL["c64"]
    # and nothing anywhere else: the hits already carry the whole norm
    assert abs(st.norm() - 1) <= 1e-5
    other = rng.integers(0, 1 << n, 4096, dtype=np.uint64)
    hit = {int(index(a, (a + b) % (1 << nb), (a + b) >> nb)) for a in range(1 << nb)}
    want = np.array([2.0 ** -8 if int(x) in hit else 0.0 for x in other])
    assert report("adder16 elsewhere", np.abs(st.amplitudes_at(other) - want), n) <= TOL["c64"]
    st.close()
    del buf
