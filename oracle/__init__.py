"""Oracle for the partitioned state-vector hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU model of what the method computes, written directly from the paper
(Fang et al., "Efficient Hierarchical State Vector Simulation of Quantum
Circuits via Acyclic Graph Partitioning", arXiv 2205.06973).  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (the HIP library and its
Python binding) never imports, links or calls anything here, and nothing
here imports the product package.

Modules
-------
statevector
    complex128 gate-at-a-time simulator (Sec. II.A-B, Sec. III.A) and a
    part-by-part executor over a partition (Sec. III.C: each part acts on the
    sub-vectors addressed by its qubits) used to pin that the hierarchical
    method reaches the gate-at-a-time result.
partition
    gate DAG (Sec. IV.A), working-set size, an exact validity check of an
    acyclic partition (Sec. IV.A conditions i-ii), the natural-order cutoff
    reference (Sec. IV.B.1) and a brute-force minimum for tiny DAGs.

Gates are plain tuples ``(name, q0, q1, params)`` with ``q1 == -1`` for a
one-qubit gate; the oracle holds its own gate definitions.
"""

from . import statevector, partition  # noqa: F401
