"""Pins of the partition oracle (Sec. IV.A model, Sec. IV.B.1 cutoff)."""

import json
import os

import pytest

from oracle import partition as op
from paper_2205_06973_amd import workloads as wl


def _gates(raw):
    return [(g[0], g[1], g[2], tuple(g[3])) for g in raw]


def test_working_set_example(golden_dir):
    with open(os.path.join(golden_dir, "paper_working_set.json")) as f:
        d = json.load(f)
    gates = _gates(d["gates"])
    assert len(op.working_set(gates, range(len(gates)))) == d["working_set"]


def test_dag_edges_by_hand():
    gates = [("h", 0, -1, ()), ("cx", 0, 1, ()), ("h", 2, -1, ()),
             ("cx", 1, 2, ()), ("h", 0, -1, ())]
    assert op.dag_edges(gates) == {(0, 1), (1, 3), (2, 3), (1, 4)}


def test_nat_examples(golden_dir):
    with open(os.path.join(golden_dir, "nat_examples.json")) as f:
        d = json.load(f)
    for case in d["cases"]:
        gates = _gates(case["gates"])
        assert op.nat_partition(gates, case["limit"]) == case["parts"]
        assert op.check_partition(8, gates, case["parts"], case["limit"]) == []
        if "brute_min" in case:
            assert op.brute_min_parts(8, gates, case["limit"]) == case["brute_min"]


def test_checker_rejects_planted_mistakes():
    gates = [("cx", 0, 1, ()), ("cx", 1, 2, ()), ("cx", 0, 1, ())]
    # valid: {g0, g1} has {0,1,2} -> needs limit 3
    assert op.check_partition(3, gates, [0, 0, 1], 3) == []
    # over the limit
    assert any("qubits >" in e for e in op.check_partition(3, gates, [0, 0, 1], 2))
    # cycle: g0, g2 in part 0, g1 in part 1: 0 -> 1 (g0->g1) and 1 -> 0 (g1->g2)
    errs = op.check_partition(3, gates, [0, 1, 0], 3)
    assert "part-graph has a cycle" in errs
    # ids not in topological order
    gates2 = [("h", 0, -1, ()), ("h", 0, -1, ())]
    assert any("earlier part" in e for e in op.check_partition(1, gates2, [1, 0], 1))
    # empty part / wrong length
    assert any("empty" in e for e in op.check_partition(1, gates2, [0, 2], 1))
    assert op.check_partition(1, gates2, [0], 1) != []


def test_is_acyclic_basic():
    assert op.is_acyclic(3, {(0, 1), (1, 2)})
    assert not op.is_acyclic(3, {(0, 1), (1, 2), (2, 0)})
    assert op.is_acyclic(2, set())


@pytest.mark.parametrize("seed", range(6))
def test_nat_valid_and_not_below_brute_force(seed):
    n = 4
    gates = wl.random_circuit(n, 7, ("h", "rz", "cx", "cz"), seed)
    for k in (2, 3):
        parts = op.nat_partition(gates, k)
        assert op.check_partition(n, gates, parts, k) == []
        assert op.num_parts(parts) >= op.brute_min_parts(n, gates, k)


def test_nat_rejects_gate_wider_than_limit():
    with pytest.raises(ValueError):
        op.nat_partition([("cx", 0, 1, ())], 1)


def test_nat_large_random_valid():
    n, gates = wl.random34(0, n=20, num_gates=400)
    for k in (3, 5, 7):
        parts = op.nat_partition(gates, k)
        assert op.check_partition(n, gates, parts, k) == []


def test_nat_padded_examples(golden_dir):
    """Multi-level first level: the padding qubits count toward every part."""
    with open(os.path.join(golden_dir, "nat_padded_examples.json")) as f:
        d = json.load(f)
    for case in d["cases"]:
        gates = _gates(case["gates"])
        got = op.nat_partition(gates, case["limit"], case["padding"])
        assert got == case["parts"]
        assert op.check_partition(8, gates, got, case["limit"], case["padding"]) == []
        if "parts_without_padding" in case:
            assert op.nat_partition(gates, case["limit"]) == case["parts_without_padding"]
    tw = d["too_wide"]
    with pytest.raises(ValueError):
        op.nat_partition(_gates([tw["gate"]]), tw["limit"], tw["padding"])


def test_checker_counts_padding():
    gates = [("h", 2, -1, ()), ("cx", 2, 3, ())]
    # {2} u {0,1} = 3 qubits; {2,3} u {0,1} = 4
    assert op.check_partition(4, gates, [0, 0], 4, padding=(0, 1)) == []
    assert any("qubits >" in e for e in op.check_partition(4, gates, [0, 0], 3, padding=(0, 1)))
    assert op.check_partition(4, gates, [0, 0], 3) == []
