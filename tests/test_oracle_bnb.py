"""Pins of the oracle's branch-and-bound (Section 4) and child fold (CPU only).

The optimum is pinned by brute force over all n! permutations and by an
independent exact solver (Gilmore-Lawler-bounded B&B that shares nothing with
the RLT2 machinery but the LAP routine).  The child fold is pinned by the
reformulation identity restricted to permutations with the fixed pair.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_03732_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("inst", [
    I.grid_n8(),
    I.grid_instance(8, 2, 4, 0.4, 1, 9, 3),
    I.dense_instance(8, 4),
    I.dense_instance(9, 5),
    I.random_instance(7, 6),
    I.random_instance(7, 7, lo=-4, hi=9),
], ids=lambda x: x.name)
def test_bnb_matches_brute_force(inst):
    F, D, B = inst.arrays()
    opt, _ = O.bruteforce(F, D, B)
    obj, perm, st = O.bnb(F, D, B, node_iters=30)
    assert obj == opt
    assert O.qap_cost(F, D, B, perm) == opt
    assert sorted(perm.tolist()) == list(range(inst.n))
    g_obj, g_perm, _ = O.glb_bnb(F, D, B)
    assert g_obj == opt
    assert O.qap_cost(F, D, B, g_perm) == opt


def test_bnb_with_forced_branching():
    """A one-iteration node cap forces deep trees; the optimum must not move."""
    inst = I.dense_instance(8, 17)
    F, D, B = inst.arrays()
    opt, _ = O.bruteforce(F, D, B)
    obj, perm, st = O.bnb(F, D, B, node_iters=1)
    assert obj == opt
    assert st["nodes"] > 1


def test_rule3_order():
    """Rule 3: lowest total interaction first, then lowest interaction with
    the facilities already placed (hand-built flows)."""
    F = np.array([[0, 5, 1, 0],
                  [5, 0, 2, 9],
                  [1, 2, 0, 0],
                  [0, 9, 0, 0]], dtype=float)
    # totals (row + column sums): f0 = 12, f1 = 32, f2 = 6, f3 = 18 -> 2 first;
    # interaction with {2}: f0 = 2, f1 = 4, f3 = 0 -> 3; with {2,3}:
    # f0 = 2, f1 = 22 -> 0; then 1.
    assert O.rule3_order(F).tolist() == [2, 3, 0, 1]


@pytest.mark.parametrize("l,s", [(0, 0), (2, 5), (5, 1)])
def test_child_fold_identity(l, s):
    inst = I.random_instance(6, 40)
    F, D, B = inst.arrays()
    da = O.DualAscent(F, D, B)
    da.run(3)
    child = da.fold(l, s)
    fi = [a for a in range(6) if a != l]
    li = [a for a in range(6) if a != s]
    for cperm in itertools.permutations(range(5)):
        perm = np.zeros(6, dtype=np.int32)
        perm[l] = s
        for a, b in enumerate(cperm):
            perm[fi[a]] = li[b]
        val = child.identity(np.array(cperm, dtype=np.int32))
        cost = O.qap_cost(F, D, B, perm)
        assert abs(val - cost) <= 1e-9 * max(1.0, abs(cost))
        # the child is a self-contained QAP: restricted F, D, folded B, offset
        Fc, Dc, Bc = child._keep
        assert O.qap_cost(Fc, Dc, Bc, np.array(cperm, dtype=np.int32)) + child.offset == cost
    assert child.LB == da.LB + da.export()[0][l, s]
    # the child's own ascent keeps the bound valid for the restricted problem
    child.run(5)
    best = min(O.qap_cost(F, D, B, np.array([s if a == l else li[cp[fi.index(a)]] for a in range(6)],
                                            dtype=np.int32))
               for cp in itertools.permutations(range(5)))
    assert child.LB <= best + 1e-9 * best


@pytest.mark.parametrize("n", [14, 16])
def test_golden_dense_optimum_fixture(n):
    """The dense optima used by the GPU B&B tests were written by
    tests/golden/make_golden.py (oracle only); both exact solvers agreed."""
    with open(os.path.join(GOLDEN, f"dense_n{n}_optimum.json")) as f:
        g = json.load(f)
    inst = I.dense_instance(n, 0)
    F, D, B = inst.arrays()
    assert g["n"] == n
    perm = np.array(g["perm"], dtype=np.int32)
    assert sorted(perm.tolist()) == list(range(n))
    assert O.qap_cost(F, D, B, perm) == g["optimum"]
    assert g["optimum"] == g["glb_bnb_optimum"] == g["rlt2_bnb_optimum"]
