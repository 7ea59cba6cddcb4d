"""Partition oracle: gate DAG, working sets, exact validity, natural cutoff.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

What it follows
---------------
* Sec. IV.A (model): vertices are the computational gates; an artificial
  entry and exit vertex per qubit carry no computation, so they are left
  implicit here.  There is an edge from a gate to the next gate that uses
  each of its qubits (the qubit dependency).  The working-set size L(V_i)
  of a part is the number of distinct qubits used by its gates (controls
  included).  A partition is valid when parts are non-empty, disjoint and
  exhaustive, (i) every part has L <= L_m, and (ii) the part-graph -- parts
  contracted to single nodes -- has no cycle.  Gates of one part run in their
  original circuit order.
* Sec. IV.B.1 (natural topological order cutoff): walk the gates in circuit
  order, growing the current part's qubit set; when adding the next gate
  would make it exceed L_m, close the part before that gate and start a new
  one.  A part of exactly L_m qubits is allowed (the limit is "not
  exceeded").
* Sec. IV.A, condition iii: the minimum number of parts; ``brute_min_parts``
  finds it by exhaustive search for DAGs of a handful of gates.
* Sec. IV.B, multi-level paragraph: a part smaller than the limit is topped
  up with qubits of the enclosing level for locality.  Reading used for a
  multi-level first level: a fixed set of padding qubits is held by every
  part, so the bound applies to the part's qubits together with the padding
  (``padding`` below; empty for a plain partition).
"""

from __future__ import annotations

import itertools
from collections import deque


def gate_qubits(gate) -> tuple[int, ...]:
    _, q0, q1, _ = gate[:4]
    if len(gate) > 4:  # three-qubit kinds carry their third qubit last
        return (q0, q1, gate[4])
    return (q0,) if q1 < 0 else (q0, q1)


def dag_edges(gates) -> set[tuple[int, int]]:
    """Edges (i, j): gate j is the next gate after gate i on a shared qubit."""
    last = {}
    edges = set()
    for j, g in enumerate(gates):
        for q in gate_qubits(g):
            if q in last:
                edges.add((last[q], j))
            last[q] = j
    return edges


def working_set(gates, members) -> set[int]:
    """L(V_i): the distinct qubits needed by the gates in ``members``."""
    qs = set()
    for i in members:
        qs.update(gate_qubits(gates[i]))
    return qs


def part_graph(gates, part_of_gate) -> set[tuple[int, int]]:
    """Cross-part edges of the DAG, contracted (Sec. IV.A, part-graph)."""
    return {(part_of_gate[i], part_of_gate[j]) for (i, j) in dag_edges(gates)
            if part_of_gate[i] != part_of_gate[j]}


def is_acyclic(num_nodes: int, edges) -> bool:
    """Kahn's algorithm: True iff the directed graph has no cycle."""
    indeg = [0] * num_nodes
    succ = [[] for _ in range(num_nodes)]
    for a, b in edges:
        succ[a].append(b)
        indeg[b] += 1
    queue = deque(v for v in range(num_nodes) if indeg[v] == 0)
    seen = 0
    while queue:
        v = queue.popleft()
        seen += 1
        for w in succ[v]:
            indeg[w] -= 1
            if indeg[w] == 0:
                queue.append(w)
    return seen == num_nodes


def check_partition(n: int, gates, part_of_gate, limit: int, padding=()) -> list[str]:
    """Every violated condition, as text; an empty list means valid.

    Conditions: one part id per gate in [0, P); every id used (non-empty
    parts); |L(V_i) u padding| <= limit; the part-graph is acyclic; and,
    because parts are executed in increasing id, every cross-part edge goes
    from a lower to a higher id (the ids are a topological order of the
    part-graph).
    """
    errors = []
    G = len(gates)
    if len(part_of_gate) != G:
        return [f"{len(part_of_gate)} part ids for {G} gates"]
    if G == 0:
        return []
    ids = [int(p) for p in part_of_gate]
    if min(ids) < 0:
        errors.append("negative part id")
        return errors
    P = max(ids) + 1
    members = [[] for _ in range(P)]
    for i, p in enumerate(ids):
        members[p].append(i)
    for p in range(P):
        if not members[p]:
            errors.append(f"part {p} is empty")
    for p in range(P):
        ws = working_set(gates, members[p]) | set(padding)
        if len(ws) > limit:
            errors.append(f"part {p} uses {len(ws)} qubits > {limit}")
    for g in gates:
        for q in gate_qubits(g):
            if not (0 <= q < n):
                errors.append(f"qubit {q} out of range for n={n}")
    pg = part_graph(gates, ids)
    if not is_acyclic(P, pg):
        errors.append("part-graph has a cycle")
    for a, b in pg:
        if a > b:
            errors.append(f"edge from part {a} to earlier part {b}")
            break
    return errors


def nat_partition(gates, limit: int, padding=()) -> list[int]:
    """Natural topological order cutoff (Sec. IV.B.1); with padding, each
    part's qubits together with the padding qubits stay within the limit."""
    part = []
    pad = set(padding)
    current: set[int] = set()
    pid = 0
    for g in gates:
        qs = set(gate_qubits(g))
        if len(qs | pad) > limit:
            raise ValueError("a gate uses more qubits than the limit")
        if current and len(current | qs | pad) > limit:
            pid += 1
            current = set()
        current |= qs
        part.append(pid)
    return part


def num_parts(part_of_gate) -> int:
    return (max(part_of_gate) + 1) if len(part_of_gate) else 0


def brute_min_parts(n: int, gates, limit: int) -> int:
    """Minimum number of parts over all valid partitions (tiny DAGs only).

    Tries P = 1, 2, ... and every assignment of gates to P labels; an
    assignment counts when the labelled parts, renumbered by a topological
    order of their part-graph, pass ``check_partition``.
    """
    G = len(gates)
    if G == 0:
        return 0
    if G > 9:
        raise ValueError("brute force is for at most 9 gates")
    for P in range(1, G + 1):
        for labels in itertools.product(range(P), repeat=G):
            if len(set(labels)) != P:
                continue
            if any(len(working_set(gates, [i for i in range(G) if labels[i] == p])) > limit
                   for p in range(P)):
                continue
            pg = part_graph(gates, list(labels))
            if is_acyclic(P, pg):
                return P
    return G
