"""Seeded synthetic circuits -- the shared input generators.

This module only draws random circuits; it holds none of the simulation's
arithmetic (no gate matrices, no partitioning), so the oracle and the HIP
path can both be fed from it.  A gate is a plain tuple
``(name, q0, q1, params)``: ``q1 == -1`` for a one-qubit gate, ``params`` a
tuple of up to three floats, and for ``cx`` q0 is the control, q1 the target.
The three-qubit kinds carry their third qubit last:
``("ccx", c0, c1, (), target)`` and ``("cswap", control, x, (), y)``.

The paper measures on QASMBench circuits (30-37 qubits, 60-5,731 gates,
Table I), which are not available here; the circuits below stand in for
them at the same scale.  Their recipes are:

* ``random_circuit``: every gate's kind uniform over ``kinds``, one-qubit
  targets uniform over the n qubits, two-qubit gates on a uniformly random
  ordered pair of distinct qubits, angles uniform on [0, 2 pi).
* ``layered_circuit``: per layer, U3(theta, phi, lambda ~ U[0, 2 pi)) on
  every qubit, then CX on a random perfect matching (odd n: one random qubit
  sits the layer out) -- the shape of the qaoa/ising families.
* ``qft_circuit``: H + controlled-phase ladder with angles pi/2^d for wire
  distance d, then the final swaps (32 H + 496 CP + 16 SWAP at n = 32).
* ``product_block_circuit``: like ``random_circuit`` but every two-qubit gate
  stays inside the even-qubit block or inside the odd-qubit block, so the
  final state factorises into an even part and an odd part.
* ``serving_stream``: Poisson arrivals of layered circuits with n ~ U{lo..hi},
  depth ~ U{lo..hi} layers, complex64 with probability 0.7 else complex128.
* ``adder_circuit``: the ripple-carry adder of Cuccaro, Draper, Kutin and
  Moulton (2004), written from its MAJ / UMA definition: on a basis input it
  maps (a, b) to (a, a + b) with the carry out in its own qubit -- a
  Toffoli-heavy circuit whose output is known exactly at any size (a 16-bit
  adder has 34 qubits).  Layout: qubit 0 is the carry-in ancilla, b_i is
  qubit 1 + 2 i, a_i is qubit 2 + 2 i, the carry out is qubit 2 nbits + 1.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * math.pi
_ONE_Q_ANGLES = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "u3": 3}
_TWO_Q = {"cx", "cz", "cp", "swap"}
_THREE_Q = {"ccx", "cswap"}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _draw_gate(rng, name: str, n: int, pair_pool=None):
    if name in _THREE_Q:
        a, b, c = rng.choice(n, size=3, replace=False)
        return (name, int(a), int(b), (), int(c))
    if name in _TWO_Q:
        if pair_pool is None:
            a, b = rng.choice(n, size=2, replace=False)
        else:
            pool = pair_pool[int(rng.integers(len(pair_pool)))]
            a, b = rng.choice(pool, size=2, replace=False)
        params = (float(rng.uniform(0.0, TWO_PI)),) if name == "cp" else ()
        return (name, int(a), int(b), params)
    q = int(rng.integers(n))
    k = _ONE_Q_ANGLES.get(name, 0)
    params = tuple(float(v) for v in rng.uniform(0.0, TWO_PI, size=k))
    return (name, q, -1, params)


def random_circuit(n: int, num_gates: int, kinds, seed: int):
    rng = _rng(seed)
    kinds = list(kinds)
    return [_draw_gate(rng, kinds[int(rng.integers(len(kinds)))], n)
            for _ in range(num_gates)]


def product_block_circuit(n: int, num_gates: int, kinds, seed: int):
    """Two-qubit gates only within the even block or within the odd block."""
    rng = _rng(seed)
    kinds = list(kinds)
    blocks = [list(range(0, n, 2)), list(range(1, n, 2))]
    blocks = [b for b in blocks if len(b) >= 2]
    return [_draw_gate(rng, kinds[int(rng.integers(len(kinds)))], n, pair_pool=blocks)
            for _ in range(num_gates)]


def layered_circuit(n: int, layers: int, seed: int):
    rng = _rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            th, ph, la = (float(v) for v in rng.uniform(0.0, TWO_PI, size=3))
            gates.append(("u3", q, -1, (th, ph, la)))
        perm = [int(v) for v in rng.permutation(n)]
        for i in range(0, n - 1, 2):
            gates.append(("cx", perm[i], perm[i + 1], ()))
    return gates


def layered_product_block_circuit(n: int, layers: int, seed: int):
    """Layered circuit whose CX matchings stay inside the even and the odd qubits."""
    rng = _rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            th, ph, la = (float(v) for v in rng.uniform(0.0, TWO_PI, size=3))
            gates.append(("u3", q, -1, (th, ph, la)))
        for block in (list(range(0, n, 2)), list(range(1, n, 2))):
            perm = [block[int(i)] for i in rng.permutation(len(block))]
            for i in range(0, len(perm) - 1, 2):
                gates.append(("cx", perm[i], perm[i + 1], ()))
    return gates


def dressed_pairs_circuit(n: int, blocks: int, seed: int, span: int = 6, dwell: int = 8):
    """Blocks of U3 on two qubits, a two-qubit gate (CX, CZ, CP or SWAP)
    on them, and U3 on both again; pairs drawn from a window of `span`
    qubits that moves up one qubit every `dwell` blocks, so a part holds
    several dressed pairs (a long dwell makes deep, dense parts)."""
    rng = _rng(seed)
    out = []
    two = ["cx", "cz", "cp", "swap"]
    for b in range(blocks):
        lo = (b // dwell) % max(1, n - span + 1)
        a, c = (int(x) + lo for x in rng.choice(span, size=2, replace=False))
        dress = lambda: [("u3", q, -1, _draw_gate(rng, "u3", n)[3]) for q in (a, c)]  # noqa: E731
        out += dress()
        g = two[int(rng.integers(len(two)))]
        out.append((g, a, c, _draw_gate(rng, g, n)[3]))
        out += dress()
    return out


def split_dressed_circuit(n: int, n_low: int, blocks: int, seed: int, span: int = 5, dwell: int = 16):
    """Two dressed-pair circuits, one on qubits [0, n_low) and one on
    [n_low, n), interleaved block by block.  No gate joins the halves, so
    the state stays a product psi_low(low bits) * psi_high(high bits) and
    every amplitude can be checked from two small simulations."""
    lo = dressed_pairs_circuit(n_low, blocks, seed, span, dwell)
    hi = dressed_pairs_circuit(n - n_low, blocks, seed + 1, span, dwell)
    shift = lambda g: (g[0], g[1] + n_low, g[2] + n_low if g[2] >= 0 else -1, g[3])  # noqa: E731
    out = []
    for b in range(blocks):  # five gates per block
        out += lo[5 * b:5 * b + 5] + [shift(g) for g in hi[5 * b:5 * b + 5]]
    return out, lo, hi


def qft_circuit(n: int):
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(("h", j, -1, ()))
        for k in range(j - 1, -1, -1):
            gates.append(("cp", k, j, (math.pi / float(1 << (j - k)),)))
    for i in range(n // 2):
        gates.append(("swap", i, n - 1 - i, ()))
    return gates


def random_basis_index(n: int, seed: int) -> int:
    return int(_rng(seed).integers(0, 1 << n, dtype=np.uint64))


def ghz_circuit(n: int):
    return [("h", 0, -1, ())] + [("cx", 0, q, ()) for q in range(1, n)]


# --- the named workloads ----------------------------------------------------

RANDOM12_KINDS = ("h", "x", "rz", "cx")
RANDOM34_KINDS = ("h", "rz", "rx", "cx", "cz")


def random12(seed: int = 0):
    """12 qubits, 200 gates over {H, X, RZ, CX}; partitioned with k = 4."""
    return 12, random_circuit(12, 200, RANDOM12_KINDS, seed)


def layered28(seed: int = 0, n: int = 28, layers: int = 40):
    """28 qubits, 40 layers of (U3 on every qubit + CX matching) = 1,680 gates."""
    return n, layered_circuit(n, layers, seed)


def qft32(seed: int = 0, n: int = 32):
    """QFT on 32 qubits applied to a seeded random basis state."""
    return n, qft_circuit(n), random_basis_index(n, seed)


def random34(seed: int = 0, n: int = 34, num_gates: int = 1000):
    """1,000 gates over {H, RZ, RX, CX, CZ}, qubits uniform (34 c64 / 33 c128)."""
    return n, random_circuit(n, num_gates, RANDOM34_KINDS, seed)


@dataclass(frozen=True)
class Request:
    arrival_s: float
    n: int
    layers: int
    dtype: str          # "c64" or "c128"
    seed: int


def serving_stream(num_requests: int, rate_per_s: float, seed: int,
                   n_range=(10, 26), layer_range=(20, 200), p_c64: float = 0.7):
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(num_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        layers = int(rng.integers(layer_range[0], layer_range[1] + 1))
        dtype = "c64" if float(rng.uniform()) < p_c64 else "c128"
        out.append(Request(t, n, layers, dtype, int(seed) * 1_000_003 + i))
    return out


def adder_circuit(nbits: int):
    """Ripple-carry adder on 2 nbits + 2 qubits (layout in the module notes)."""
    a = lambda i: 2 + 2 * i  # noqa: E731
    b = lambda i: 1 + 2 * i  # noqa: E731
    carry = lambda i: 0 if i == 0 else a(i - 1)  # noqa: E731
    gates = []
    for i in range(nbits):  # MAJ(carry_i, b_i, a_i)
        gates += [("cx", a(i), b(i), ()), ("cx", a(i), carry(i), ()),
                  ("ccx", carry(i), b(i), (), a(i))]
    gates.append(("cx", a(nbits - 1), 2 * nbits + 1, ()))
    for i in reversed(range(nbits)):  # UMA(carry_i, b_i, a_i)
        gates += [("ccx", carry(i), b(i), (), a(i)), ("cx", a(i), carry(i), ()),
                  ("cx", carry(i), b(i), ())]
    return 2 * nbits + 2, gates
