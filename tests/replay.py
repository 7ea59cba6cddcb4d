"""Host replay of compiled part descriptors (test helper, not a simulator path).

Given the descriptors that ``hs_plan_part_descriptors`` reports for a part
(the tile's qubits, the load / stage / store layouts and the register
operations), apply them to a numpy complex128 vector exactly as their
documented meaning says, so the part compiler can be checked against the
oracle on a machine without a GPU.  Written from the header's description of
the descriptors, not from the kernel source.
"""

from __future__ import annotations

import numpy as np


def _tile_index(pos, m: int, coords: np.ndarray) -> np.ndarray:
    t = np.zeros_like(coords)
    for c in range(m):
        t |= ((coords >> c) & 1) << int(pos[c])
    return t


def _insert_zero_bits(tile: int, qubits) -> int:
    b = tile
    for q in sorted(int(x) for x in qubits):
        b = ((b >> q) << (q + 1)) | (b & ((1 << q) - 1))
    return b


def _apply_ops(R: np.ndarray, ops: np.ndarray, rb: int, nthr: int) -> None:
    """R: complex vector over coordinates; coordinate = thr | j << log2(nthr)."""
    V = R.reshape(1 << rb, nthr)  # row j = register j of every thread
    for op in ops:
        kind, b0, b1 = int(op[0]), int(op[1]), int(op[2])
        c = op[3:]
        J = np.arange(1 << rb)
        if kind in (0, 1, 4):
            lo = J[(J >> b0) & 1 == 0]
            hi = lo | (1 << b0)
            x, y = V[lo].copy(), V[hi].copy()
            if kind == 0:
                u = [complex(c[0], c[1]), complex(c[2], c[3]), complex(c[4], c[5]),
                     complex(c[6], c[7])]
            elif kind == 1:
                u = [c[0], c[1], c[2], c[3]]
            else:
                u = [0, 1, 1, 0]
            V[lo] = u[0] * x + u[1] * y
            V[hi] = u[2] * x + u[3] * y
        elif kind == 2:
            one = (J >> b0) & 1 == 1
            V[~one] *= complex(c[0], c[1])
            V[one] *= complex(c[2], c[3])
        elif kind == 3:
            V[(J >> b0) & 1 == 1] *= complex(c[0], c[1])
        elif kind == 5:
            src = J[((J >> b0) & 1 == 1) & ((J >> b1) & 1 == 0)]
            dst = src | (1 << b1)
            V[src], V[dst] = V[dst].copy(), V[src].copy()
        elif kind in (6, 7):
            both = ((J >> b0) & 1 == 1) & ((J >> b1) & 1 == 1)
            V[both] *= -1.0 if kind == 6 else complex(c[0], c[1])
        elif kind == 8:
            src = J[((J >> b0) & 1 == 1) & ((J >> b1) & 1 == 0)]
            dst = src ^ (1 << b0) ^ (1 << b1)
            V[src], V[dst] = V[dst].copy(), V[src].copy()
        elif kind == 9:  # dense 4x4, quad index = bit b0 + 2 bit b1
            M = (c[0:32:2] + 1j * c[1:32:2]).reshape(4, 4)
            base = J[((J >> b0) & 1 == 0) & ((J >> b1) & 1 == 0)]
            rows = [base, base | (1 << b0), base | (1 << b1), base | (1 << b0) | (1 << b1)]
            X = [V[r].copy() for r in rows]
            for i in range(4):
                V[rows[i]] = sum(M[i, k] * X[k] for k in range(4))
        else:
            raise ValueError(f"unknown op kind {kind}")


def replay_part(psi: np.ndarray, n: int, hdr, ent, ops) -> dict:
    """Apply one compiled part to psi in place; returns layout facts for checks."""
    m, lb, wb, rb, ne = (int(v) for v in hdr[:5])
    tq = [int(v) for v in hdr[8:8 + m]]
    nthr = 1 << (lb + wb)
    coords = np.arange(1 << m, dtype=np.int64)
    tidx = [_tile_index(ent[e, :16], m, coords) for e in range(ne)]
    for e in range(ne):
        assert sorted(tidx[e].tolist()) == list(range(1 << m)), "layout is not a bijection"
        if e > 0 and not ent[e, 18]:
            assert np.array_equal(tidx[e], tidx[e - 1]), "layout changed without a transition"
    # global offset of every tile index
    t_all = np.arange(1 << m, dtype=np.int64)
    goff = np.zeros(1 << m, dtype=np.int64)
    for i, q in enumerate(tq):
        goff |= ((t_all >> i) & 1) << q
    for tile in range(1 << (n - m)):
        base = _insert_zero_bits(tile, tq)
        addr = base + goff
        tile_vec = psi[addr]
        R = tile_vec[tidx[0]].copy()                          # load layout
        for e in range(1, ne):
            if ent[e, 18]:                                    # re-layout
                tv = np.empty_like(R)
                tv[tidx[e - 1]] = R
                R = tv[tidx[e]]
            _apply_ops(R, ops[ent[e, 16]:ent[e, 17]], rb, nthr)
        tv = np.empty_like(R)
        tv[tidx[ne - 1]] = R                                  # store layout
        psi[addr] = tv
    lanes_load = [int(ent[0, c]) for c in range(lb)]
    lanes_store = [int(ent[ne - 1, c]) for c in range(lb)]
    return {"m": m, "lb": lb, "wb": wb, "rb": rb, "tq": tq,
            "load_lane_qubits": [tq[t] for t in lanes_load],
            "store_lane_qubits": [tq[t] for t in lanes_store]}


def replay_plan(plan, n: int, psi0: np.ndarray, dtype: str = "c64", mode: str = "part_lds"):
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    facts = []
    for p in range(plan.num_parts):
        hdr, ent, ops = plan.part_descriptors(p, dtype, mode)
        facts.append(replay_part(psi, n, hdr, ent, ops))
    return psi, facts
