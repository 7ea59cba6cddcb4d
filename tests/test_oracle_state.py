"""Pins of the state-vector oracle against things other than itself.

* the matrices and the X action printed in Sec. II.A (golden fixture);
* the pair structure of Sec. III.A / Fig. 1 (golden fixture);
* the gather map of the worked example in Sec. III.C (golden fixture);
* rotations rebuilt as matrix exponentials of the paper's Pauli matrices
  (scipy.linalg.expm), U3 as RZ(phi) RY(theta) RZ(lambda) up to its phase;
* brute force: every gate embedded into a dense 2^n x 2^n matrix by explicit
  basis-index loops (two-qubit gates assembled from projectors and the
  paper's X/Z), multiplied out and applied, for n <= 6;
* closed forms: GHZ, H on every qubit, QFT of a basis state, QFT of any
  state = sqrt(N) * numpy.fft.ifft;
* invariants: norm preservation, inverse round trip, Alg. 1 over any valid
  partition equals the gate-at-a-time result.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import partition as op
from oracle import statevector as sv
from paper_2205_06973_amd import workloads as wl


def _mat(entries):
    return np.array([[complex(re, im) for re, im in row] for row in entries])


@pytest.fixture(scope="module")
def paper_gates(golden_dir):
    with open(os.path.join(golden_dir, "paper_gates.json")) as f:
        d = json.load(f)
    return {"x": _mat(d["x"]), "y": _mat(d["y"]), "z": _mat(d["z"]),
            "h": _mat(d["h_times_sqrt2"]) / math.sqrt(2.0)}


def test_paper_matrices(paper_gates):
    for name in ("x", "y", "z", "h"):
        np.testing.assert_allclose(sv.gate_matrix_1q(name), paper_gates[name], atol=0)


def test_x_swaps_amplitudes():
    # Sec. II.A: X (a0, a1) = (a1, a0)
    psi = np.array([0.6, 0.8j], dtype=np.complex128)
    sv.apply_gate(psi, ("x", 0, -1, ()))
    np.testing.assert_array_equal(psi, np.array([0.8j, 0.6]))


def test_unitarity_all_kinds():
    rng = np.random.default_rng(1)
    for name in sv.ONE_QUBIT:
        p = tuple(rng.uniform(0, 2 * math.pi, size=3))
        u = sv.gate_matrix_1q(name, p)
        np.testing.assert_allclose(u @ u.conj().T, np.eye(2), atol=1e-15)


def test_rotations_are_exponentials_of_paper_paulis(paper_gates):
    X, Y, Z = paper_gates["x"], paper_gates["y"], paper_gates["z"]
    for th in (0.0, 0.3, 1.7, 4.0, 6.1):
        np.testing.assert_allclose(sv.gate_matrix_1q("rx", (th,)),
                                   scipy.linalg.expm(-0.5j * th * X), atol=1e-14)
        np.testing.assert_allclose(sv.gate_matrix_1q("ry", (th,)),
                                   scipy.linalg.expm(-0.5j * th * Y), atol=1e-14)
        np.testing.assert_allclose(sv.gate_matrix_1q("rz", (th,)),
                                   scipy.linalg.expm(-0.5j * th * Z), atol=1e-14)
        # P(l) = e^{il/2} RZ(l)
        np.testing.assert_allclose(sv.gate_matrix_1q("p", (th,)),
                                   np.exp(0.5j * th) * scipy.linalg.expm(-0.5j * th * Z),
                                   atol=1e-14)
    rng = np.random.default_rng(2)
    for _ in range(5):
        th, ph, la = rng.uniform(0, 2 * math.pi, size=3)
        rz = lambda a: scipy.linalg.expm(-0.5j * a * Z)  # noqa: E731
        ry = scipy.linalg.expm(-0.5j * th * Y)
        want = np.exp(0.5j * (ph + la)) * (rz(ph) @ ry @ rz(la))
        np.testing.assert_allclose(sv.gate_matrix_1q("u3", (th, ph, la)), want, atol=1e-14)
    # S = P(pi/2), T = P(pi/4); H = (X + Z)/sqrt(2)
    np.testing.assert_allclose(sv.gate_matrix_1q("s"), sv.gate_matrix_1q("p", (math.pi / 2,)),
                               atol=1e-15)
    np.testing.assert_allclose(sv.gate_matrix_1q("t"), sv.gate_matrix_1q("p", (math.pi / 4,)),
                               atol=1e-15)
    np.testing.assert_allclose(paper_gates["h"], (X + Z) / math.sqrt(2), atol=1e-15)


def test_pair_structure_fig1(golden_dir):
    with open(os.path.join(golden_dir, "paper_h3_pairs.json")) as f:
        d = json.load(f)
    n = d["n"]
    for q, pairs in d["pairs"].items():
        q = int(q)
        assert len(pairs) == 2 ** (n - 1)
        for a, b in pairs:
            assert b - a == d["stride"][str(q)] == 2 ** q
            # H on qubit q couples exactly a and b: the image of e_a lives on {a, b}
            for src in (a, b):
                psi = sv.basis_state(n, src)
                sv.apply_gate(psi, ("h", q, -1, ()))
                assert set(np.flatnonzero(np.abs(psi) > 0)) == {a, b}


def test_gather_map_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "paper_gather_example.json")) as f:
        d = json.load(f)
    addr = sv.gather_addresses(d["n"], d["part_qubits"])
    np.testing.assert_array_equal(addr, np.array(d["gather"]))
    # disjoint and collectively exhaustive (Sec. III.C)
    assert sorted(addr.ravel().tolist()) == list(range(2 ** d["n"]))


@pytest.mark.parametrize("n,part", [(4, [0, 1]), (5, [4, 1]), (6, [0, 2, 5]), (3, [0, 1, 2]),
                                    (7, [6])])
def test_split_by_part_explicit_indices(n, part):
    """The sub-vector view against explicit bit arithmetic: row r, slot j
    holds the amplitude whose index has bit b of r on the b-th smallest outer
    qubit and bit b of j on the b-th smallest part qubit; merging undoes it."""
    rng = np.random.default_rng(n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    mat = sv.split_by_part(psi, n, part)
    qs = sorted(part)
    outer = [q for q in range(n) if q not in qs]
    for r in range(1 << len(outer)):
        for j in range(1 << len(qs)):
            i = sum(((r >> b) & 1) << q for b, q in enumerate(outer))
            i |= sum(((j >> b) & 1) << q for b, q in enumerate(qs))
            assert mat[r, j] == psi[i]
    np.testing.assert_array_equal(sv.merge_by_part(mat, n, part), psi)


# --- brute force ------------------------------------------------------------

def _embed(n, qubits, small):
    """2^n x 2^n matrix of ``small`` acting on ``qubits`` (bit k of the small
    index = value of qubits[k]); identity elsewhere.  Explicit index loops."""
    N = 1 << n
    big = np.zeros((N, N), dtype=np.complex128)
    others = [q for q in range(n) if q not in qubits]
    for i in range(N):
        for j in range(N):
            if any(((i >> q) & 1) != ((j >> q) & 1) for q in others):
                continue
            si = sum(((i >> q) & 1) << k for k, q in enumerate(qubits))
            sj = sum(((j >> q) & 1) << k for k, q in enumerate(qubits))
            big[i, j] = small[si, sj]
    return big


def _brute_gate(n, gate, paper_gates):
    name, q0, q1, p = gate
    P0 = np.diag([1.0, 0.0]).astype(np.complex128)
    P1 = np.diag([0.0, 1.0]).astype(np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    if q1 < 0:
        return _embed(n, [q0], sv.gate_matrix_1q(name, p))
    # small index: bit 0 = q0, bit 1 = q1  ->  kron(op on q1, op on q0)
    if name == "cx":
        small = np.kron(I2, P0) + np.kron(paper_gates["x"], P1)
    elif name == "cz":
        small = np.kron(I2, P0) + np.kron(paper_gates["z"], P1)
    elif name == "cp":
        small = np.kron(I2, P0) + np.kron(np.diag([1.0, np.exp(1j * p[0])]), P1)
    elif name == "swap":
        cx01 = np.kron(I2, P0) + np.kron(paper_gates["x"], P1)
        cx10 = np.kron(P0, I2) + np.kron(P1, paper_gates["x"])
        small = cx01 @ cx10 @ cx01
    else:
        raise ValueError(name)
    return _embed(n, [q0, q1], small)


ALL_KINDS = sv.ONE_QUBIT + sv.TWO_QUBIT


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (5, 4), (6, 5)])
def test_brute_force_dense_product(n, seed, paper_gates):
    kinds = ALL_KINDS if n >= 2 else sv.ONE_QUBIT
    gates = wl.random_circuit(n, 25, kinds, seed)
    # an arbitrary (normalised) input makes every column of U count
    rng = np.random.default_rng(seed)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    U = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        U = _brute_gate(n, g, paper_gates) @ U
    want = U @ psi0
    got = sv.simulate(n, gates, psi0)
    np.testing.assert_allclose(got, want, atol=1e-13, rtol=0)


def test_two_qubit_argument_order(paper_gates):
    # CX(c, t) must not be confused with CX(t, c): |c=1, t=0> -> |1, 1>
    n = 3
    for c, t in [(0, 2), (2, 0), (1, 2), (2, 1)]:
        psi = sv.basis_state(n, 1 << c)
        sv.apply_gate(psi, ("cx", c, t, ()))
        assert abs(psi[(1 << c) | (1 << t)] - 1) < 1e-15
        psi = sv.basis_state(n, 1 << t)
        sv.apply_gate(psi, ("cx", c, t, ()))
        assert abs(psi[1 << t] - 1) < 1e-15


# --- closed forms -----------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 10, 14])
def test_ghz_closed_form(n):
    psi = sv.simulate(n, wl.ghz_circuit(n))
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, want, atol=1e-15)


def test_hadamard_all_uniform():
    n = 9
    psi = sv.simulate(n, [("h", q, -1, ()) for q in range(n)])
    np.testing.assert_allclose(psi, np.full(1 << n, 2 ** (-n / 2)), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9])
def test_qft_of_basis_state_closed_form(n):
    N = 1 << n
    for x in sorted({0, 1, N - 1, (0x5A5A5 % N), (N // 3)}):
        psi = sv.simulate(n, wl.qft_circuit(n), x)
        y = np.arange(N)
        want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
        np.testing.assert_allclose(psi, want, atol=1e-13)


@pytest.mark.parametrize("n", [4, 8, 11])
def test_qft_equals_scaled_ifft(n):
    rng = np.random.default_rng(n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    got = sv.simulate(n, wl.qft_circuit(n), psi0)
    want = math.sqrt(1 << n) * np.fft.ifft(psi0)
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_qft32_gate_count():
    n, gates, _ = wl.qft32(0)
    names = [g[0] for g in gates]
    assert (names.count("h"), names.count("cp"), names.count("swap")) == (32, 496, 16)


# --- invariants -------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_norm_and_inverse_round_trip(seed):
    n = 10
    gates = wl.random_circuit(n, 300, ALL_KINDS, seed)
    psi = sv.simulate(n, gates, 0)
    assert abs(sv.norm(psi) - 1.0) < 1e-12
    back = sv.simulate(n, sv.inverse_circuit(gates), psi)
    want = sv.basis_state(n, 0)
    np.testing.assert_allclose(back, want, atol=1e-12)


@pytest.mark.parametrize("seed,k", [(0, 2), (1, 3), (2, 4), (3, 5)])
def test_alg1_equals_gate_at_a_time(seed, k):
    n = 7
    gates = wl.random_circuit(n, 60, ALL_KINDS, seed)
    parts = op.nat_partition(gates, k)
    assert op.check_partition(n, gates, parts, k) == []
    want = sv.simulate(n, gates, 3)
    got = sv.simulate_alg1(n, gates, parts, 3)
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_alg1_detects_wrong_part_order():
    # Running the parts of a valid partition in the wrong order changes the
    # result: the check above is not vacuous.
    n = 4
    gates = [("h", 0, -1, ()), ("cx", 0, 1, ()), ("h", 1, -1, ()), ("cx", 1, 2, ())]
    parts = op.nat_partition(gates, 2)
    assert max(parts) >= 1
    flipped = [max(parts) - p for p in parts]
    want = sv.simulate(n, gates)
    got = sv.simulate_alg1(n, gates, flipped)
    assert np.max(np.abs(got - want)) > 1e-3


def test_product_block_factorises():
    n = 10
    gates = wl.product_block_circuit(n, 120, ("h", "rz", "rx", "cx", "cz"), 7)
    for g in gates:
        if g[2] >= 0:
            assert g[1] % 2 == g[2] % 2
    psi = sv.simulate(n, gates)
    ev = [g for g in gates if g[1] % 2 == 0]
    od = [g for g in gates if g[1] % 2 == 1]
    ren = lambda g: (g[0], g[1] // 2, g[2] // 2 if g[2] >= 0 else -1, g[3])  # noqa: E731
    pe = sv.simulate(n // 2, [ren(g) for g in ev])
    po = sv.simulate(n // 2, [ren(g) for g in od])
    idx = np.arange(1 << n)
    ie = sum(((idx >> (2 * b)) & 1) << b for b in range(n // 2))
    io = sum(((idx >> (2 * b + 1)) & 1) << b for b in range(n // 2))
    np.testing.assert_allclose(psi, pe[ie] * po[io], atol=1e-13)


def test_state_bytes(golden_dir):
    with open(os.path.join(golden_dir, "paper_state_bytes.json")) as f:
        d = json.load(f)
    for n, gib in d["table1_gib"].items():
        assert (2 ** int(n)) * d["bytes_per_amplitude_c128"] == gib * 2 ** 30
    assert sv.basis_state(4).itemsize == d["bytes_per_amplitude_c128"]


# ---- three-qubit gates (applied whole by the oracle) -------------------------------

def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("a,b,t", [(0, 1, 2), (3, 0, 1), (2, 3, 0)])
def test_ccx_is_h_ccz_h(a, b, t):
    """Toffoli = H on the target, a phase of -1 where all three bits are 1
    (a diagonal built from the index bits), H on the target."""
    n = 4
    psi = _rand_state(n, 11 + a)
    want = psi.copy()
    sv.apply_gate(want, ("h", t, -1, ()))
    idx = np.arange(1 << n)
    ccz = np.where(((idx >> a) & (idx >> b) & (idx >> t) & 1) == 1, -1.0, 1.0)
    want *= ccz
    sv.apply_gate(want, ("h", t, -1, ()))
    got = psi.copy()
    sv.apply_gate(got, ("ccx", a, b, (), t))
    np.testing.assert_allclose(got, want, atol=1e-14)


@pytest.mark.parametrize("c,x,y", [(0, 1, 2), (2, 3, 0), (1, 0, 3)])
def test_cswap_is_cx_ccx_cx(c, x, y):
    n = 4
    psi = _rand_state(n, 21 + c)
    want = psi.copy()
    for g in (("cx", y, x, ()), ("ccx", c, x, (), y), ("cx", y, x, ())):
        sv.apply_gate(want, g)
    got = psi.copy()
    sv.apply_gate(got, ("cswap", c, x, (), y))
    np.testing.assert_allclose(got, want, atol=1e-14)
    sv.apply_gate(got, ("cswap", c, x, (), y))  # self-inverse
    np.testing.assert_allclose(got, psi, atol=1e-14)


def _adder_index(nb, a, b, carry=0):
    x = carry << (2 * nb + 1)
    for i in range(nb):
        x |= ((a >> i) & 1) << (2 + 2 * i)
        x |= ((b >> i) & 1) << (1 + 2 * i)
    return x


def test_adder_closed_form():
    """The ripple-carry adder maps |a, b> to |a, a + b> (carry in its qubit)."""
    nb = 3
    n, gates = wl.adder_circuit(nb)
    for a in range(1 << nb):
        for b in range(1 << nb):
            psi = sv.simulate(n, gates, _adder_index(nb, a, b))
            s = a + b
            assert abs(psi[_adder_index(nb, a, s % (1 << nb), s >> nb)] - 1) < 1e-12
