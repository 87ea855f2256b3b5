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


@pytest.mark.parametrize("m", [8, 13, 28, 40, 64, 65, 129, 300, 1024])
def test_lap_value_equals_scipy(m):
    rng = np.random.default_rng(7 * m)
    for trial in range(6):
        M = rng.integers(0, 100, size=(m, m)).astype(float) if trial % 2 else rng.random((m, m))
        th, *_ = O.lap(M)
        r, c = linear_sum_assignment(M)
        opt = M[r, c].sum()
        assert abs(th - opt) <= 1e-9 * max(1.0, abs(opt))


def test_lap_refuses_beyond_its_size_limit():
    with pytest.raises(ValueError):
        O.lap(np.zeros((1025, 1025)))


@pytest.mark.parametrize("m", [3, 9, 28, 200])
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


def test_lap_zero_matrix():
    """All-zero matrix: the column reduction matches column 0 to row 0 (every
    column proposes row 0, the lowest column wins); each other row's search
    ends at once on the lowest unmatched column (ties prefer unmatched
    columns): m - 1 steps, identity assignment, all duals zero."""
    for m in (1, 4, 28):
        th, u, v, rc, pi, steps = O.lap(np.zeros((m, m)))
        assert th == 0.0 and steps == m - 1
        assert rc.tolist() == list(range(m))
        assert not u.any() and not v.any()


def test_lap_hand_worked_2x2():
    """M = [[1,2],[3,4]], worked by hand through the specified steps.
    Column reduction: v = (1, 2), both columns propose row 0, column 0 wins;
    value starts at 1 + 2 = 3.  Row 1: s = (3-0-1, 4-0-2) = (2, 2), the tie
    goes to the unmatched column 1, delta = 2: u1 = 2, value 5; column 1 is
    free, so row 1 takes it."""
    th, u, v, rc, pi, steps = O.lap(np.array([[1.0, 2.0], [3.0, 4.0]]))
    assert th == 5.0
    assert u.tolist() == [0.0, 2.0]
    assert v.tolist() == [1.0, 2.0]
    assert rc.tolist() == [0, 1]
    assert steps == 1
    assert not pi.any()


def test_lap_hand_worked_3x3_augmenting_path():
    """M = [[0,1,5],[0,4,5],[5,5,0]] by hand.
    Column reduction: v = (0, 1, 0); columns 0 and 1 propose row 0 (column 0
    wins), column 2 proposes row 2; value starts at 1.  Row 1: s = (0, 3, 5),
    j* = 0 (matched to row 0), delta 0; scanning row 0 gives column 1
    s = (1-0)-1 = 0 < 3 (via column 0); j* = 1 is free, delta 0.  Path:
    column 1 <- row 0, column 0 <- row 1.  Result row0->col1, row1->col0,
    row2->col2, theta = 1, u = 0, v = (0, 1, 0)."""
    M = np.array([[0.0, 1.0, 5.0], [0.0, 4.0, 5.0], [5.0, 5.0, 0.0]])
    th, u, v, rc, pi, steps = O.lap(M)
    assert th == 1.0
    assert rc.tolist() == [1, 0, 2]
    assert u.tolist() == [0.0, 0.0, 0.0]
    assert v.tolist() == [0.0, 1.0, 0.0]
    assert steps == 2
