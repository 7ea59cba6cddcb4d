"""complex128 gate-at-a-time state-vector simulator -- the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

What it follows
---------------
* Sec. II.B: the state of an n-qubit system is a vector of 2^n complex
  amplitudes (16 bytes each, i.e. complex128); simulating a circuit applies
  each gate of the sequence, in order, to that vector.
* Sec. III.A and the Fig. 1 caption: amplitudes are indexed little-endian,
  so bit q of the index is the value of qubit q; a one-qubit gate on qubit i
  pairs the amplitudes whose indices differ only in bit i (stride s = 2^i)
  and multiplies each pair by the 2x2 gate matrix -- 2^(n-1) independent
  matrix-vector products per gate.
* Sec. II.A: the matrices of X, Y, Z and H are the ones printed there.  The
  paper names CX and SWAP without matrices and uses rotation/phase gates
  only through its benchmark circuits; the readings used for RX, RY, RZ, P,
  U3, S, T, CX, CZ, CP and SWAP are the standard OpenQASM-2 ones, listed in
  the design notes (rotation RZ keeps its global phase:
  RZ(t) = diag(e^{-it/2}, e^{it/2})).
* Sec. II.A: probabilities are |amplitude|^2 (the paper writes alpha^2).
* Sec. III.C: ``simulate_alg1`` applies a given partition part by part: the
  state is viewed as one sub-vector of 2^w amplitudes (the part's qubits)
  per setting of the other qubits, the part's gates act on every sub-vector,
  and the view is undone.  The inner slots take the part's qubits in
  ascending global order, which matches the worked example of Sec. III.C
  (S0 = {q1, q0} -> in_sv[q1, q0]).

Two-qubit gates are written by what they do to amplitudes, so no 4x4
basis-ordering convention is needed:
  CX(c, t):  for indices with bit c = 1, swap the pair differing in bit t;
  CZ(a, b):  negate amplitudes with bit a = bit b = 1;
  CP(l)(a,b): multiply amplitudes with bit a = bit b = 1 by e^{il};
  SWAP(a, b): exchange amplitudes with (bit a, bit b) = (1, 0) and (0, 1).
Three-qubit gates (the paper decomposes gates on more qubits, Sec. III.A
footnote; the oracle applies them whole, by definition), written as
(name, q0, q1, params, q2):
  CCX(a, b, t): for indices with bit a = bit b = 1, swap the pair differing
                in bit t;
  CSWAP(c, x, y): for indices with bit c = 1, exchange amplitudes with
                (bit x, bit y) = (1, 0) and (0, 1).

Everything is float64 / complex128 numpy; no blocking, fusion or reordering.
"""

from __future__ import annotations

import math

import numpy as np

ONE_QUBIT = ("h", "x", "y", "z", "s", "t", "rx", "ry", "rz", "p", "u3")
TWO_QUBIT = ("cx", "cz", "cp", "swap")
THREE_QUBIT = ("ccx", "cswap")


def gate_matrix_1q(name: str, params=()) -> np.ndarray:
    """2x2 complex128 matrix of a one-qubit gate (Sec. II.A; readings above)."""
    p = tuple(float(v) for v in params)
    if name == "h":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    if name == "x":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if name == "y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if name == "z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if name == "s":
        return np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    if name == "t":
        return np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)
    if name == "rx":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "ry":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if name == "rz":
        return np.array([[np.exp(-0.5j * p[0]), 0], [0, np.exp(0.5j * p[0])]],
                        dtype=np.complex128)
    if name == "p":
        return np.array([[1, 0], [0, np.exp(1j * p[0])]], dtype=np.complex128)
    if name == "u3":
        th, ph, la = p[0], p[1], p[2]
        c, s = math.cos(th / 2), math.sin(th / 2)
        return np.array([[c, -np.exp(1j * la) * s],
                         [np.exp(1j * ph) * s, np.exp(1j * (ph + la)) * c]],
                        dtype=np.complex128)
    raise ValueError(f"not a one-qubit gate: {name!r}")


def num_qubits_of(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.ndim != 1 or (1 << n) != psi.size:
        raise ValueError("state must be a 1-D vector of length 2^n")
    return n


def basis_state(n: int, x: int = 0) -> np.ndarray:
    """|x> as complex128 (Sec. II.B); x = 0 is |0...0>."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def apply_1q(psi: np.ndarray, q: int, u: np.ndarray) -> None:
    """In place: the 2^(n-1) scoped 2x2 products of Sec. III.A on qubit q.

    Viewing the vector as (high, bit q, low) puts the two members of every
    pair (index with bit q = 0, the same index with bit q = 1) at [:, 0, :]
    and [:, 1, :].
    """
    v = psi.reshape(-1, 2, 1 << q)
    a0 = v[:, 0, :].copy()
    a1 = v[:, 1, :].copy()
    v[:, 0, :] = u[0, 0] * a0 + u[0, 1] * a1
    v[:, 1, :] = u[1, 0] * a0 + u[1, 1] * a1


def _view2(psi: np.ndarray, n: int, a: int, b: int) -> tuple[np.ndarray, bool]:
    """View psi as [high, bit hi, mid, bit lo, low] for qubits a != b.

    Returns the view and whether ``a`` is the higher of the two qubits.
    """
    hi, lo = (a, b) if a > b else (b, a)
    v = psi.reshape(1 << (n - hi - 1), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    return v, a > b


def apply_2q(psi: np.ndarray, name: str, a: int, b: int, params=()) -> None:
    """In place: CX(control a, target b), CZ, CP(lambda), SWAP on qubits a, b."""
    n = num_qubits_of(psi)
    v, a_is_hi = _view2(psi, n, a, b)

    def sl(bit_a: int, bit_b: int):
        # index into the 5-D view with the bits of qubits a and b fixed
        if a_is_hi:
            return (slice(None), bit_a, slice(None), bit_b, slice(None))
        return (slice(None), bit_b, slice(None), bit_a, slice(None))

    if name == "cx":
        t0 = v[sl(1, 0)].copy()
        v[sl(1, 0)] = v[sl(1, 1)]
        v[sl(1, 1)] = t0
    elif name == "cz":
        v[sl(1, 1)] *= -1.0
    elif name == "cp":
        v[sl(1, 1)] *= np.exp(1j * float(params[0]))
    elif name == "swap":
        t0 = v[sl(1, 0)].copy()
        v[sl(1, 0)] = v[sl(0, 1)]
        v[sl(0, 1)] = t0
    else:
        raise ValueError(f"not a two-qubit gate: {name!r}")


def apply_3q(psi: np.ndarray, name: str, a: int, b: int, c: int) -> None:
    """In place: CCX(a, b -> c) or CSWAP(a; b <-> c), by index arithmetic."""
    n = num_qubits_of(psi)
    idx = np.arange(1 << n, dtype=np.int64)

    def bit(q):
        return (idx >> q) & 1

    if name == "ccx":
        sel = idx[(bit(a) == 1) & (bit(b) == 1) & (bit(c) == 0)]
        other = sel | (1 << c)
    elif name == "cswap":
        sel = idx[(bit(a) == 1) & (bit(b) == 1) & (bit(c) == 0)]
        other = sel ^ (1 << b) ^ (1 << c)
    else:
        raise ValueError(f"not a three-qubit gate: {name!r}")
    tmp = psi[sel].copy()
    psi[sel] = psi[other]
    psi[other] = tmp


def check_gate(n: int, gate) -> None:
    name, q0, q1, _ = gate[:4]
    if name in THREE_QUBIT:
        q2 = gate[4] if len(gate) > 4 else -1
        if not all(0 <= q < n for q in (q0, q1, q2)) or len({q0, q1, q2}) != 3:
            raise ValueError(f"bad three-qubit gate {gate!r} for n={n}")
        return
    if name in ONE_QUBIT:
        if not (0 <= q0 < n) or q1 != -1:
            raise ValueError(f"bad one-qubit gate {gate!r} for n={n}")
    elif name in TWO_QUBIT:
        if not (0 <= q0 < n and 0 <= q1 < n) or q0 == q1:
            raise ValueError(f"bad two-qubit gate {gate!r} for n={n}")
    else:
        raise ValueError(f"unknown gate {name!r}")


def apply_gate(psi: np.ndarray, gate) -> None:
    name, q0, q1, params = gate[:4]
    n = num_qubits_of(psi)
    check_gate(n, gate)
    if name in ONE_QUBIT:
        apply_1q(psi, q0, gate_matrix_1q(name, params))
    elif name in THREE_QUBIT:
        apply_3q(psi, name, q0, q1, gate[4])
    else:
        apply_2q(psi, name, q0, q1, params)


def simulate(n: int, gates, init=0) -> np.ndarray:
    """Apply ``gates`` in circuit order to |init> (an int) or to a given vector.

    Sec. II.B: the simulation applies each gate of the sequence to the state.
    """
    if isinstance(init, np.ndarray):
        psi = np.array(init, dtype=np.complex128, copy=True)
        if psi.size != (1 << n):
            raise ValueError("initial vector has the wrong length")
    else:
        psi = basis_state(n, int(init))
    for g in gates:
        apply_gate(psi, g)
    return psi


def probabilities(psi: np.ndarray) -> np.ndarray:
    """|a|^2 per amplitude (Sec. II.A, read as the squared modulus)."""
    return psi.real * psi.real + psi.imag * psi.imag


def norm(psi: np.ndarray) -> float:
    """Sum of |a|^2 over the whole state (1 for a normalised state)."""
    return float(math.fsum(probabilities(psi).tolist())) if psi.size <= (1 << 16) \
        else float(np.sum(probabilities(psi), dtype=np.float64))


def inverse_gate(gate):
    """The gate whose matrix is the adjoint of ``gate``'s (for round trips)."""
    name, q0, q1, p = gate[:4]
    p = tuple(p)
    if name in ("h", "x", "y", "z", "cx", "cz", "swap", "ccx", "cswap"):
        return gate
    if name == "s":
        return ("p", q0, q1, (-math.pi / 2,))
    if name == "t":
        return ("p", q0, q1, (-math.pi / 4,))
    if name in ("rx", "ry", "rz", "p", "cp"):
        return (name, q0, q1, (-p[0],))
    if name == "u3":
        # U3(t, f, l)^dagger = U3(-t, -l, -f)
        return ("u3", q0, q1, (-p[0], -p[2], -p[1]))
    raise ValueError(name)


def inverse_circuit(gates):
    return [inverse_gate(g) for g in reversed(list(gates))]


# ---------------------------------------------------------------------------
# Hierarchical execution over a partition (Sec. III.C), by tensor views
# ---------------------------------------------------------------------------

def _part_perm(n: int, part_qubits) -> list[int]:
    """Axis order that views a (2,)*n state tensor as (outer qubits, part qubits).

    numpy's row-major reshape of the 2^n vector puts qubit q on axis n-1-q
    (the last axis is the least significant bit).  After this permutation
    the leading axes are the qubits outside the part, highest first, and the
    trailing axes the part's qubits, highest first; flattening the two groups
    gives (row r, column j) with bit b of r = the b-th smallest outer qubit
    and bit b of j = the b-th smallest part qubit -- the inner-slot order of
    the worked example of Sec. III.C (S0 = {q1, q0} -> in_sv[q1, q0]).
    """
    part = sorted(int(q) for q in part_qubits)
    outer = [q for q in range(n) if q not in part]
    return [n - 1 - q for q in reversed(outer)] + [n - 1 - q for q in reversed(part)]


def split_by_part(psi: np.ndarray, n: int, part_qubits) -> np.ndarray:
    """The state as a (2^(n-w), 2^w) matrix: row r holds the 2^w amplitudes of
    outer setting r (Sec. III.C: the sub-vectors addressed by the part's
    qubits, one per setting of the others; disjoint and exhaustive)."""
    w = len(set(int(q) for q in part_qubits))
    t = np.asarray(psi).reshape((2,) * n).transpose(_part_perm(n, part_qubits))
    return np.ascontiguousarray(t).reshape(1 << (n - w), 1 << w)


def merge_by_part(mat: np.ndarray, n: int, part_qubits) -> np.ndarray:
    """Inverse of split_by_part: the matrix of sub-vectors back to the 2^n state."""
    perm = _part_perm(n, part_qubits)
    t = np.asarray(mat).reshape((2,) * n).transpose(np.argsort(perm))
    return np.ascontiguousarray(t).reshape(1 << n)


def gather_addresses(n: int, part_qubits) -> np.ndarray:
    """Index map of the split: entry [r, j] is the state index whose amplitude
    lands in inner slot j for outer setting r."""
    return split_by_part(np.arange(1 << n, dtype=np.int64), n, part_qubits)


def simulate_alg1(n: int, gates, part_of_gate, init=0) -> np.ndarray:
    """Hierarchical simulation over a given partition (Sec. III.C).

    Parts are applied one after another in increasing part id (the ids must
    already be a topological order of the part-graph).  A part with qubit set
    S (w qubits) acts only on the sub-vectors addressed by S: the state is
    split into its 2^(n-w) sub-vectors of 2^w amplitudes, the part's gates --
    in circuit order (Sec. IV.A) and renamed to inner slots -- are applied to
    every sub-vector, and the sub-vectors are merged back.  Applying a gate on
    slot b to the flattened (row, slot) matrix acts on bit b of every row at
    once, so all outer settings are handled in one call per gate.
    """
    psi = simulate(n, [], init)
    parts = {}
    for gi, p in enumerate(part_of_gate):
        parts.setdefault(int(p), []).append(gi)
    for p in sorted(parts):
        part_gates = [gates[i] for i in parts[p]]
        qubits = sorted({q for g in part_gates for q in (g[1], g[2]) + tuple(g[4:5]) if q >= 0})
        slot = {q: j for j, q in enumerate(qubits)}
        renamed = [(g[0], slot[g[1]], slot[g[2]] if g[2] >= 0 else -1, g[3])
                   + ((slot[g[4]],) if len(g) > 4 else ()) for g in part_gates]
        rows = split_by_part(psi, n, qubits).reshape(-1)
        for g in renamed:
            apply_gate(rows, g)
        psi = merge_by_part(rows, n, qubits)
    return psi
