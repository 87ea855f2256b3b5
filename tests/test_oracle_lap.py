"""Pins of the oracle's Hungarian LAP solver (CPU only).

The LAP is the building block of every stage of the three-stage solution of
LRLT2 (Section 2.3, "LAP Solution").  Its optimum is pinned by brute force over
all m! assignments and by an independent library routine; its duals by the
complementary slackness conditions of Eq. (compslack); the specified choice of
duals by hand-worked examples.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import oracle as O


def _brute(M):
    m = M.shape[0]
    best = np.inf
    for perm in itertools.permutations(range(m)):
        best = min(best, sum(M[i, perm[i]] for i in range(m)))
    return best


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_lap_value_equals_brute_force(m):
    rng = np.random.default_rng(100 + m)
    for trial in range(25):
        if trial % 3 == 0:
            M = rng.integers(0, 4, size=(m, m)).astype(float)      # heavy ties
        elif trial % 3 == 1:
            M = rng.normal(size=(m, m))                            # negative entries too
        else:
            M = rng.random((m, m)) * 1e3
        th, u, v, rc, pi, _ = O.lap(M)
        opt = _brute(M)
        assert abs(th - opt) <= 1e-9 * max(1.0, abs(opt))
        assert sorted(rc.tolist()) == list(range(m))


@pytest.mark.parametrize("m", [8, 13, 28, 40, 64])
def test_lap_value_equals_scipy(m):
    rng = np.random.default_rng(7 * m)
    for trial in range(6):
        M = rng.integers(0, 100, size=(m, m)).astype(float) if trial % 2 else rng.random((m, m))
        th, *_ = O.lap(M)
        r, c = linear_sum_assignment(M)
        opt = M[r, c].sum()
        assert abs(th - opt) <= 1e-9 * max(1.0, abs(opt))


@pytest.mark.parametrize("m", [3, 9, 28])
def test_lap_duals_complementary_slackness(m):
    """Dual feasibility u_i + v_j <= M_ij and pi = 0 on the assignment
    (Eq. compslack); the dual objective equals the LAP value."""
    rng = np.random.default_rng(m)
    for trial in range(10):
        M = rng.random((m, m)) * 10.0 if trial % 2 else rng.integers(0, 3, (m, m)).astype(float)
        th, u, v, rc, pi, _ = O.lap(M)
        scale = max(1.0, np.abs(M).max())
        assert pi.min() >= -1e-12 * scale
        assert np.abs(pi[rc, np.arange(m)]).max() <= 1e-12 * scale
        primal = M[rc, np.arange(m)].sum()
        assert abs(th - primal) <= 1e-12 * max(1.0, abs(primal)) * m
        assert abs((u.sum() + v.sum()) - primal) <= 1e-12 * max(1.0, abs(primal)) * m


def test_lap_rank_one_closed_form():
    """M_jq = a_j b_q: the optimum is the minimum scalar product, sorted a
    against reverse-sorted b (rearrangement inequality).  This is exactly the
    Y-LAP of the first iteration, whose value builds the Gilmore-Lawler bound
    (Section 5.1)."""
    rng = np.random.default_rng(3)
    for m in (2, 5, 13, 29):
        a = rng.integers(0, 100, size=m).astype(float)
        b = rng.integers(0, 100, size=m).astype(float)
        th, *_ = O.lap(np.outer(a, b))
        closed = float(np.sort(a) @ np.sort(b)[::-1])
        assert th == closed


def test_lap_zero_matrix_one_step_per_row():
    """All-zero matrix: every row's search ends at once on the lowest unmatched
    column (ties prefer unmatched columns), so m rows take m steps, the
    assignment is the identity and all duals stay zero."""
    for m in (1, 4, 28):
        th, u, v, rc, pi, steps = O.lap(np.zeros((m, m)))
        assert th == 0.0 and steps == m
        assert rc.tolist() == list(range(m))
        assert not u.any() and not v.any()


def test_lap_hand_worked_2x2():
    """M = [[1,2],[3,4]], worked by hand through the specified steps.
    Row 0: minv = (1, 2) -> j* = 0, delta = 1, u0 = 1, col 0 <- row 0.
    Row 1: minv = (3, 4) -> j* = 0 (matched), delta = 3, u1 = 3; scan row 0:
    s_1 = (2 - 1) - 0 = 1 is not strictly below minv_1 = 1, so column 1 keeps
    its link to the root; j* = 1, delta = 1: u1 = 4, u0 = 2, v0 = -1.
    Column 1 is free: the path is just column 1, so row 1 takes column 1 and
    row 0 keeps column 0.  theta = 1 + 3 + 1 = 5."""
    th, u, v, rc, pi, steps = O.lap(np.array([[1.0, 2.0], [3.0, 4.0]]))
    assert th == 5.0
    assert u.tolist() == [2.0, 4.0]
    assert v.tolist() == [-1.0, 0.0]
    assert rc.tolist() == [0, 1]
    assert steps == 3
    assert not pi.any()


def test_lap_hand_worked_3x3_augmenting_path():
    """M = [[0,1,5],[0,4,5],[5,5,0]] by hand.
    Row 0: minv = (0,1,5), j* = 0 free: col0 <- row0, delta 0.
    Row 1: minv = (0,4,5): j* = 0 (matched, delta 0); scan row 0: s = (1,5)
    for cols 1,2 improves col 1 to 1 (via col 0); j* = 1 free, delta = 1:
    u1 = 1, u0 = 1, v0 = -1.  Path: col1 <- row0, col0 <- row1.
    Row 2: minv = (6, 5, 0) -> j* = 2 free, delta 0.
    Result: row0->col1, row1->col0, row2->col2, theta = 1."""
    M = np.array([[0.0, 1.0, 5.0], [0.0, 4.0, 5.0], [5.0, 5.0, 0.0]])
    th, u, v, rc, pi, steps = O.lap(M)
    assert th == 1.0
    assert rc.tolist() == [1, 0, 2]
    assert u.tolist() == [1.0, 1.0, 0.0]
    assert v.tolist() == [-1.0, 0.0, 0.0]
    assert steps == 4
