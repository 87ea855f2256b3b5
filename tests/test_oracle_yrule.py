"""Pins of the oracle's y-pair rule (Eq. da:yrule1, Algorithm 1 step 4a), CPU only.

The rule hands a fraction phi_y of the difference between the reduced costs
of the complementary y pair (i,j,p,q) / (j,i,q,p) from the larger to the
smaller one, and moves the pair's Lagrange multiplier u by the same amount.
What fixes it, independently of the oracle's own code:
  * worked examples whose results were computed by hand (below);
  * the pair's sum is conserved (a zero-sum move keeps every permutation's
    cost, Section 2.3);
  * the pair's difference shrinks by the factor (1 - 2 phi_y): phi_y = 1/2
    makes the pair equal, phi_y = 0 changes nothing, phi_y = 1 swaps it;
  * entries with i = j or p = q, and the x and z levels, are not touched;
  * the multiplier moves opposite to the reduced cost (S-form costs are
    C - u), so u changes by exactly the cost given away, zero-sum per pair.
Sum and difference together determine a linear rule on (a, b), so a no-op,
swapped phi_y / (1 - phi_y), or a wrong partner index fails here.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_03732_amd import instances as I


def _state(n, Y, phiy, seed=0):
    """An oracle state holding the given dense Y, random X and Z, and
    parameters (FULL kz, ky, kx, phi) with the y-pair share phiy."""
    rng = np.random.default_rng(seed)
    F = rng.integers(0, 9, (n, n)).astype(float)
    D = rng.integers(0, 9, (n, n)).astype(float)
    Bm = np.zeros((n, n))
    X = rng.random((n, n))
    Z = rng.random((n,) * 6)
    params = (5.0 / 6.0, 1.0, 1.0, 1.0 / 5.0, phiy)
    da = O.DualAscent.from_arrays(F, D, Bm, params, 3.5, X, Y, Z)
    return da, X, Z


def _pairs(n):
    for i, j in itertools.combinations(range(n), 2):
        for p, q in itertools.permutations(range(n), 2):
            yield (i, j, p, q), (j, i, q, p)


def test_worked_example_by_hand():
    """n = 3, phi_y = 0.3.  Values worked by hand from Eq. da:yrule1:
    a' = 0.7 a + 0.3 b, b' = 0.7 b + 0.3 a, u_a += 0.3 (a - b)."""
    n = 3
    Y = np.zeros((n,) * 4)
    # (entry a, entry b, a, b, a', b', change of u_a)
    worked = [
        ((0, 1, 0, 1), (1, 0, 1, 0), 10.0, 4.0, 8.2, 5.8, 1.8),
        ((0, 1, 2, 0), (1, 0, 0, 2), 0.0, 5.0, 1.5, 3.5, -1.5),
        ((0, 2, 1, 2), (2, 0, 2, 1), 7.0, 7.0, 7.0, 7.0, 0.0),
        ((1, 2, 0, 1), (2, 1, 1, 0), -2.0, 8.0, 1.0, 5.0, -3.0),
        ((1, 2, 2, 0), (2, 1, 0, 2), 100.0, 0.0, 70.0, 30.0, 30.0),
    ]
    for a, b, va, vb, *_ in worked:
        Y[a], Y[b] = va, vb
    da, _, _ = _state(n, Y, 0.3)
    da.track()
    da.yequal()
    _, Y2, _ = da.export()
    _, U = da.multipliers()
    for a, b, va, vb, ea, eb, du in worked:
        assert Y2[a] == pytest.approx(ea, rel=1e-14, abs=1e-13), (a, Y2[a], ea)
        assert Y2[b] == pytest.approx(eb, rel=1e-14, abs=1e-13), (b, Y2[b], eb)
        assert U[a] == pytest.approx(du, rel=1e-14, abs=1e-13)
        assert U[b] == pytest.approx(-du, rel=1e-14, abs=1e-13)
    # every other pair held zeros and stays zero
    untouched = {x for w in worked for x in w[:2]}
    for a, b in _pairs(n):
        if a not in untouched:
            assert Y2[a] == 0.0 and Y2[b] == 0.0 and U[a] == 0.0 and U[b] == 0.0


@pytest.mark.parametrize("phiy", [0.0, 0.3, 0.5, 0.8, 1.0])
def test_pair_sum_kept_and_difference_scaled(phiy):
    """Random dense Y at n = 5: for every complementary pair the sum is
    kept and the difference scales by (1 - 2 phi_y); the x and z levels, the
    bound and the entries with i = j or p = q do not move."""
    n = 5
    rng = np.random.default_rng(7)
    Y = rng.normal(scale=50.0, size=(n,) * 4)
    da, X, Z = _state(n, Y, phiy, seed=1)
    da.track()
    da.yequal()
    X2, Y2, Z2 = da.export()
    _, U = da.multipliers()
    assert da.LB == 3.5
    assert np.array_equal(X2, X) and np.array_equal(Z2, Z)
    scale = np.abs(Y).max()
    seen = np.zeros(Y.shape, dtype=bool)
    for a, b in _pairs(n):
        ya, yb = Y[a], Y[b]
        na, nb = Y2[a], Y2[b]
        assert abs((na + nb) - (ya + yb)) <= 4e-15 * scale
        assert abs((na - nb) - (1.0 - 2.0 * phiy) * (ya - yb)) <= 4e-15 * scale
        # the multiplier takes what the cost gives away, zero-sum per pair
        assert abs(U[a] - (ya - na)) <= 4e-15 * scale
        assert abs(U[a] + U[b]) <= 4e-15 * scale
        seen[a] = seen[b] = True
    if phiy == 0.5:
        for a, b in _pairs(n):
            assert Y2[a] == Y2[b]
    if phiy == 0.0:
        assert np.array_equal(Y2, Y)
    if phiy == 1.0:
        for a, b in _pairs(n):
            assert Y2[a] == Y[b] and Y2[b] == Y[a]
    # i = j or p = q: no y variable, never paired, never changed
    assert np.array_equal(Y2[~seen], Y[~seen]) and np.all(U[~seen] == 0.0)


def test_rule_on_an_ascent_state_keeps_the_identity_and_pairs_up():
    """On a real mid-ascent state of an asymmetric instance (where the rule
    moves cost), after the Z-LAPs of an iteration t >= 1: the rule keeps the
    reformulation identity for every permutation and leaves each pair at
    its mean (phi_y = 1/2, the FULL preset)."""
    inst = I.random_instance(6, 21)  # asymmetric F and D, B != 0
    F, D, Bm = inst.arrays()
    n = inst.n
    da = O.DualAscent(F, D, Bm)
    da.run(3)
    da.sweep()
    da.zphase()
    _, Y, _ = da.export()
    moved = max(abs(Y[a] - Y[b]) for a, b in _pairs(n))
    assert moved > 1e-3  # the pairs differ before the rule
    perms = list(itertools.permutations(range(n)))[::37]
    before = [da.identity(np.array(p)) for p in perms]
    da.yequal()
    _, Y2, _ = da.export()
    for a, b in _pairs(n):
        assert Y2[a] == Y2[b]
        assert abs(Y2[a] - 0.5 * (Y[a] + Y[b])) <= 1e-12 * max(1.0, abs(Y[a]) + abs(Y[b]))
    after = [da.identity(np.array(p)) for p in perms]
    for x, y in zip(before, after):
        assert abs(x - y) <= 1e-9 * max(1.0, abs(x))
