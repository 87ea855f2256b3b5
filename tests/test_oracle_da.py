"""Pins of the oracle's F1 RLT2 dual ascent (CPU only).

What fixes the method's results independently of the oracle itself:
  * iteration 0 (v = 0) gives the Gilmore-Lawler bound (Section 5.1); the
    bound has a closed form by the rearrangement inequality, computed here
    with numpy sorting and scipy's LAP solver;
  * weak duality, Eq. (lgduality): every bound is <= the QAP optimum
    (brute force over all n! permutations);
  * Theorem 1: the bound sequence is non-decreasing;
  * every ascent move and LAP extraction preserves the reformulation
    identity cost(sigma) = LB + picked reduced costs, and leaves the reduced
    costs non-negative (dual feasibility of the LAPs, Eq. compslack);
  * f = 0 reduces the QAP to a plain LAP on b.
The trajectory values LB_t for t >= 1 are not printed anywhere in the paper
(parity unpinned); they are covered only by the invariants above.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import oracle as O
from paper_1710_03732_amd import instances as I


def glb_closed_form(F, D, B):
    n = F.shape[0]
    L = np.zeros((n, n))
    for i in range(n):
        fi = np.sort(np.delete(F[i], i))
        for p in range(n):
            dp = np.sort(np.delete(D[p], p))[::-1]
            L[i, p] = B[i, p] + F[i, i] * D[p, p] + float(fi @ dp)
    r, c = linear_sum_assignment(L)
    return float(L[r, c].sum())


def brute_opt(F, D, B):
    n = F.shape[0]
    best = np.inf
    for perm in itertools.permutations(range(n)):
        p = np.array(perm)
        best = min(best, float((B[np.arange(n), p]).sum() + (F * D[np.ix_(p, p)]).sum()))
    return best


INSTANCES = [
    I.grid_n8(),
    I.grid_instance(7, 2, 4, 0.4, 1, 9, 5),
    I.dense_instance(7, 11),
    I.random_instance(6, 21),                       # asymmetric, diagonals, B != 0
    I.random_instance(5, 22, lo=-3, hi=5),          # negative data
]


@pytest.mark.parametrize("inst", INSTANCES, ids=lambda x: x.name)
def test_iteration0_is_gilmore_lawler(inst):
    F, D, B = inst.arrays()
    da = O.DualAscent(F, D, B)
    da.run(1)
    assert da.LB == glb_closed_form(F, D, B)


@pytest.mark.parametrize("inst", INSTANCES[1:], ids=lambda x: x.name)
def test_bound_below_optimum_and_monotone(inst):
    F, D, B = inst.arrays()
    opt = brute_opt(F, D, B)
    da = O.DualAscent(F, D, B)
    da.run(40)
    tr = da.trace()
    assert len(tr) >= 1
    assert np.all(np.diff(tr) >= -1e-9 * max(1.0, abs(opt)))          # Theorem 1
    assert np.all(tr <= opt + 1e-9 * max(1.0, abs(opt)))              # Eq. lgduality
    assert da.UB >= opt
    if da.proven():
        assert da.UB == opt


def test_grid_n8_bound_and_optimum():
    inst = I.grid_n8()
    F, D, B = inst.arrays()
    opt, _ = O.bruteforce(F, D, B)
    assert opt == brute_opt(F, D, B)
    da = O.DualAscent(F, D, B)
    da.run(50)
    tr = da.trace()
    assert np.all(np.diff(tr) >= -1e-9)
    assert tr[-1] <= opt
    # the bound climbs well above the Gilmore-Lawler bound
    assert tr[-1] > tr[0]


def _check_identity(da, F, D, B, perms, tol=1e-9):
    for perm in perms:
        val = da.identity(perm)
        cost = O.qap_cost(F, D, B, perm)
        assert abs(val - cost) <= tol * max(1.0, abs(cost)), (perm, val, cost)
    mins = da.min_entries()
    scale = max(1.0, np.abs(F).max() * np.abs(D).max())
    assert mins.min() >= -1e-9 * scale


@pytest.mark.parametrize("inst", [I.random_instance(5, 3), I.grid_instance(6, 2, 3, 0.4, 1, 9, 4),
                                  I.random_instance(6, 8, lo=0, hi=20)], ids=lambda x: x.name)
def test_reformulation_identity_every_phase(inst):
    """Each move (sweep, Z/Y/X extraction, y-pair rule) preserves the
    identity for every permutation, and reduced costs stay >= 0."""
    F, D, B = inst.arrays()
    n = F.shape[0]
    perms = [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
    da = O.DualAscent(F, D, B)
    _check_identity(da, F, D, B, perms)
    for t in range(4):
        if t >= 1:
            da.sweep()
            _check_identity(da, F, D, B, perms)
        da.zphase()
        _check_identity(da, F, D, B, perms)
        if t >= 1:
            da.yequal()
            _check_identity(da, F, D, B, perms)
        da.yphase()
        _check_identity(da, F, D, B, perms)
        da.xphase()
        _check_identity(da, F, D, B, perms)


def test_identity_random_perms_n9_many_iterations():
    inst = I.grid_instance(9, 3, 3, 0.4, 1, 10, 2)
    F, D, B = inst.arrays()
    rng = np.random.default_rng(0)
    perms = [rng.permutation(9).astype(np.int32) for _ in range(300)]
    da = O.DualAscent(F, D, B)
    da.run(30)
    _check_identity(da, F, D, B, perms)
    opt = brute_opt(F, D, B)
    assert da.LB <= opt + 1e-9 * opt


def test_zero_flows_reduce_to_lap_on_b():
    rng = np.random.default_rng(5)
    n = 7
    F = np.zeros((n, n))
    D = rng.integers(0, 50, size=(n, n)).astype(float)
    B = rng.integers(0, 50, size=(n, n)).astype(float)
    da = O.DualAscent(F, D, B)
    da.run(3)
    r, c = linear_sum_assignment(B)
    opt = float(B[r, c].sum())
    assert da.trace()[0] == opt
    assert da.proven() and da.UB == opt
    assert da.t == 1  # certificate fires after the first iteration


def test_thread_count_does_not_change_results():
    inst = I.grid_instance(9, 3, 3, 0.4, 1, 10, 9)
    F, D, B = inst.arrays()
    O.set_threads(1)
    a = O.DualAscent(F, D, B)
    a.run(6)
    O.set_threads(4)
    b = O.DualAscent(F, D, B)
    b.run(6)
    O.set_threads(O.max_threads())
    assert np.array_equal(a.trace(), b.trace())
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)


def _orbit_members(i, j, k, p, q, r):
    return [(a, b, c, x, y, z) for (a, x), (b, y), (c, z) in
            itertools.permutations([(i, p), (j, q), (k, r)])]


@pytest.mark.parametrize("kz", [5.0 / 6.0, 1.0])
def test_sweep_moves_z_mass_only_inside_orbits(kz):
    """With ky = kx = 0 the sweep only redistributes z slack among the six
    symmetric variables of each orbit (Eq. rlt2:con3, Type 1 rule): each
    orbit's total is conserved, kz = 1 gives (S - pi_e) / 5, and the FULL
    choice kz = 5/6, phi = 1/5 equalises the orbit at S / 6."""
    n = 6
    rng = np.random.default_rng(12)
    F = rng.integers(0, 9, size=(n, n)).astype(float)
    D = rng.integers(0, 9, size=(n, n)).astype(float)
    B = np.zeros((n, n))
    X = rng.random((n, n))
    Y = rng.random((n,) * 4)
    Z = rng.random((n,) * 6)
    da = O.DualAscent.from_arrays(F, D, B, (kz, 0.0, 0.0, 0.2, 0.5), 0.0, X, Y, Z)
    da.sweep()
    X1, Y1, Z1 = da.export()
    assert np.array_equal(X1, X)  # okx = 1 keeps x costs
    for (i, j, k) in itertools.combinations(range(n), 3):
        for (p, q, r) in itertools.permutations(range(n), 3):
            mem = _orbit_members(i, j, k, p, q, r)
            old = np.array([Z[m] for m in mem])
            new = np.array([Z1[m] for m in mem])
            S = old.sum()
            assert abs(new.sum() - S) <= 1e-12 * S
            if kz == 1.0:
                assert np.allclose(new, (S - old) / 5.0, rtol=1e-13, atol=0)
            else:
                assert np.allclose(new, S / 6.0, rtol=1e-13, atol=0)


def test_sweep_pushes_x_and_y_slack_down():
    """Type 2 and 3 rules (Eqs. da:rule2, da:rule3): with kz = 0, ky = kx = 1
    the z level starts at zero, the y and x levels are emptied, and each
    orbit receives, per member e, phi times its partners' shares
    pi_y(P1P2(f)) / (n-2) + pi_x(P1(f)) / ((n-1)(n-2))."""
    n = 6
    rng = np.random.default_rng(13)
    F = rng.integers(0, 9, size=(n, n)).astype(float)
    D = rng.integers(0, 9, size=(n, n)).astype(float)
    X = rng.random((n, n))
    Y = rng.random((n,) * 4)
    Z = np.zeros((n,) * 6)
    da = O.DualAscent.from_arrays(F, D, np.zeros((n, n)), (0.0, 1.0, 1.0, 0.2, 0.5), 0.0, X, Y, Z)
    da.sweep()
    X1, Y1, Z1 = da.export()
    assert not X1.any()
    for (i, j, k) in [(0, 1, 2), (1, 3, 5), (0, 4, 5)]:
        for (p, q, r) in [(0, 1, 2), (5, 3, 1), (2, 0, 4)]:
            mem = _orbit_members(i, j, k, p, q, r)
            share = np.array([Y[a, b, x, y] / (n - 2) + X[a, x] / ((n - 1) * (n - 2))
                              for (a, b, c, x, y, z) in mem])
            for e, m in enumerate(mem):
                expect = 0.2 * (share.sum() - share[e])
                assert abs(Z1[m] - expect) <= 1e-13 * share.sum()


@pytest.mark.parametrize("inst", [I.grid_instance(7, 2, 4, 0.4, 1, 9, 1), I.random_instance(6, 77)],
                         ids=lambda x: x.name)
def test_sampled_iteration_paths_match_full_oracle(inst):
    """The reduced paths used at n = 30/42 (iteration 0 without the zero z
    level, single iteration-1 tiles built entry by entry) reproduce the full
    dense oracle exactly."""
    F, D, B = inst.arrays()
    n = inst.n
    full = O.DualAscent(F, D, B)
    full.run(1)
    X0, Y0, _ = full.export()
    red = O.Iter0XY(F, D, B)
    Xr, Yr = red.xy()
    assert red.LB == full.LB and red.UB == full.UB
    assert np.array_equal(Xr, X0) and np.array_equal(Yr, Y0)
    full.sweep()
    full.zphase()
    _, _, Z1 = full.export()
    for (i, j, p, q) in [(0, 1, 0, 1), (2, 0, 3, 1), (n - 1, n - 2, 0, n - 1), (1, 3, 4, 2)]:
        M, pi, th = red.tile1(i, j, p, q)
        ks = [k for k in range(n) if k not in (i, j)]
        rs = [r for r in range(n) if r not in (p, q)]
        assert np.array_equal(pi, np.array([[Z1[i, j, k, p, q, r] for r in rs] for k in ks]))


@pytest.mark.parametrize("inst", [I.grid_instance(9, 3, 3, 0.4, 1, 10, 2), I.dense_instance(8, 3),
                                  I.random_instance(7, 5)], ids=lambda x: x.name)
def test_tracked_multipliers_reproduce_the_bound(inst):
    """The F1 transfers are multiplier updates (Eq. ch4:proof:2 per sweep,
    Eq. da:yrule1 per y-pair rule).  Tracked from zero they are zero-sum over
    every orbit and pair, and the Lagrangian relaxation LRLT2(u, v) solved
    from scratch on the costs (b, C - u, -v) gives at least the F1 bound
    (Eq. ch4:proof:4, applied at every iteration)."""
    F, D, Bm = inst.arrays()
    n = inst.n
    da = O.DualAscent(F, D, Bm)
    da.track()
    da.run(25)
    V, U = da.multipliers()
    scale = max(1.0, np.abs(V).max())
    for (i, j, k) in itertools.combinations(range(n), 3):
        for (p, q, r) in [(0, 1, 2), (n - 1, 0, 3), (2, n - 2, 1)]:
            tot = sum(V[m] for m in _orbit_members(i, j, k, p, q, r))
            assert abs(tot) <= 1e-9 * scale
    for i in range(n):
        for j in range(n):
            if i != j:
                assert np.all(np.abs(U[i, j] + U[j, i].T)[~np.eye(n, dtype=bool)] <= 1e-9 * scale)
    s = O.DualAscent.from_multipliers(F, D, Bm, O.FULL, V, U)
    s.run(1)
    assert s.LB >= da.LB - 1e-9 * max(1.0, abs(da.LB))
    assert s.LB <= O.bruteforce(F, D, Bm)[0] + 1e-9


# ---- HALF scheme (Section 5): only the Z-LAPs of tiles with i < j ----------

def _lower(m):
    """A member index tuple (i, j, k, p, q, r) is lower when i > j."""
    return m[0] > m[1]


@pytest.mark.parametrize("inst", INSTANCES[1:], ids=lambda x: x.name)
def test_half_bound_below_optimum_and_monotone(inst):
    F, D, B = inst.arrays()
    opt = brute_opt(F, D, B)
    da = O.DualAscent(F, D, B, O.HALF)
    da.run(40)
    tr = da.trace()
    assert np.all(np.diff(tr) >= -1e-9 * max(1.0, abs(opt)))          # Theorem 1
    assert np.all(tr <= opt + 1e-9 * max(1.0, abs(opt)))              # Eq. lgduality
    assert da.UB >= opt
    if da.proven():
        assert da.UB == opt


@pytest.mark.parametrize("inst", [I.random_instance(5, 3), I.grid_instance(6, 2, 3, 0.4, 1, 9, 4),
                                  I.random_instance(6, 8, lo=0, hi=20)], ids=lambda x: x.name)
def test_half_reformulation_identity_every_phase(inst):
    """HALF moves (sweep with the upper/lower shares, the Z-LAPs of tiles
    with i < j only, y-pair rule, Y/X extraction) keep the identity for every
    permutation and reduced costs >= 0 (a share that gives away more or less
    than the giver's g breaks the identity); lower z costs stay exactly 0."""
    F, D, B = inst.arrays()
    n = F.shape[0]
    perms = [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
    lower = np.zeros((n,) * 6, dtype=bool)
    for i in range(n):
        lower[i, :i] = True
    da = O.DualAscent(F, D, B, O.HALF)
    for t in range(4):
        if t >= 1:
            da.sweep()
            _check_identity(da, F, D, B, perms)
            assert not da.export()[2][lower].any()
        da.zphase()
        _check_identity(da, F, D, B, perms)
        assert not da.export()[2][lower].any()
        if t >= 1:
            da.yequal()
        da.yphase()
        da.xphase()
        _check_identity(da, F, D, B, perms)


def test_half_sweep_shares_by_hand():
    """One HALF sweep from upper z slack and y/x slack: every upper member
    keeps (1 - 2/3) of its own z slack and receives half of each other upper
    member's g and a third of each lower member's g, where
    g = kz*pi_z + pi_y(P1P2)/(n-2) + pi_x(P1)/((n-1)(n-2)) and lower members
    have pi_z = 0, kz = 1; lower members end at 0; the orbit total is
    conserved."""
    n = 6
    rng = np.random.default_rng(21)
    F = rng.integers(0, 9, size=(n, n)).astype(float)
    D = rng.integers(0, 9, size=(n, n)).astype(float)
    X = rng.random((n, n))
    Y = rng.random((n,) * 4)
    Z = rng.random((n,) * 6)
    for i in range(n):
        Z[i, :i] = 0.0  # lower members hold no z cost
    da = O.DualAscent.from_arrays(F, D, np.zeros((n, n)), O.HALF, 0.0, X, Y, Z)
    da.sweep()
    X1, Y1, Z1 = da.export()
    valid_y = np.ones((n,) * 4, dtype=bool)
    for a in range(n):
        valid_y[a, a] = False
        valid_y[:, :, a, a] = False
    assert not X1.any() and not Y1[valid_y].any()  # ky = kx = 1 empty the x and y levels
    for (i, j, k) in [(0, 1, 2), (1, 3, 5), (0, 4, 5), (2, 3, 4)]:
        for (p, q, r) in [(0, 1, 2), (5, 3, 1), (2, 0, 4), (4, 5, 3)]:
            mem = _orbit_members(i, j, k, p, q, r)
            g = []
            for m in mem:
                a, b, c, x, y, z = m
                kz = 1.0 if _lower(m) else 2.0 / 3.0
                g.append(kz * Z[m] + Y[a, b, x, y] / (n - 2) + X[a, x] / ((n - 1) * (n - 2)))
            ups = [e for e, m in enumerate(mem) if not _lower(m)]
            lows = [e for e, m in enumerate(mem) if _lower(m)]
            assert ups == [0, 1, 3] and lows == [2, 4, 5]
            total = 0.0
            for e in ups:
                expect = Z[mem[e]] / 3.0 + 0.5 * sum(g[f] for f in ups if f != e) + sum(g[f] for f in lows) / 3.0
                assert abs(Z1[mem[e]] - expect) <= 1e-13 * max(1.0, expect)
                total += Z1[mem[e]]
            for e in lows:
                assert Z1[mem[e]] == 0.0
            assert abs(total - sum(g) - sum(Z[mem[e]] / 3.0 for e in ups)) <= 1e-12 * total


def test_half_keeps_up_with_full_on_the_grid():
    """The paper's claim for HALF: about the bound of solving every Z-LAP
    for half the Z-LAPs. On the 2x4 grid instance both reach within 1 % of
    the optimum in 60 iterations."""
    inst = I.grid_n8()
    F, D, B = inst.arrays()
    opt = brute_opt(F, D, B)
    full = O.DualAscent(F, D, B)
    half = O.DualAscent(F, D, B, O.HALF)
    full.run(60)
    half.run(60)
    assert half.LB <= opt and full.LB <= opt
    assert half.LB >= 0.99 * opt and full.LB >= 0.99 * opt


def test_half_refuses_nonzero_lower_costs_and_tracking():
    n = 5
    rng = np.random.default_rng(3)
    F = rng.integers(0, 9, size=(n, n)).astype(float)
    D = rng.integers(0, 9, size=(n, n)).astype(float)
    Z = np.zeros((n,) * 6)
    Z[3, 1, 0, 0, 1, 2] = 1.0  # a lower member with cost
    with pytest.raises(ValueError):
        O.DualAscent.from_arrays(F, D, np.zeros((n, n)), O.HALF, 0.0, np.zeros((n, n)), np.zeros((n,) * 4), Z)
    da = O.DualAscent(F, D, None, O.HALF)
    with pytest.raises(Exception):
        da.track()


@pytest.mark.parametrize("inst", [I.grid_instance(7, 2, 4, 0.4, 1, 9, 1), I.random_instance(6, 77)],
                         ids=lambda x: x.name)
def test_half_sampled_tiles_match_full_half_oracle(inst):
    """The single-tile path under HALF (used at n = 30) reproduces the dense
    HALF oracle's iteration-1 upper tiles exactly and refuses lower ones."""
    F, D, B = inst.arrays()
    n = inst.n
    full = O.DualAscent(F, D, B, O.HALF)
    full.run(1)
    X0, Y0, _ = full.export()
    red = O.Iter0XY(F, D, B, O.HALF)
    Xr, Yr = red.xy()
    assert red.LB == full.LB and np.array_equal(Xr, X0) and np.array_equal(Yr, Y0)
    full.sweep()
    full.zphase()
    _, _, Z1 = full.export()
    for (i, j, p, q) in [(0, 1, 0, 1), (0, 2, 3, 1), (n - 2, n - 1, 0, n - 1), (1, 3, 4, 2)]:
        M, pi, th = red.tile1(i, j, p, q)
        ks = [k for k in range(n) if k not in (i, j)]
        rs = [r for r in range(n) if r not in (p, q)]
        assert np.array_equal(pi, np.array([[Z1[i, j, k, p, q, r] for r in rs] for k in ks]))
    with pytest.raises(ValueError):
        red.tile1(1, 0, 0, 1)


# ---- two-phase variant F2 (Section 3.4): pool the orbit slacks, re-solve ----

def _pool_state(n, orbits):
    """A fresh state whose z slacks are the given orbits' six values (in the
    canonical member order) and zero elsewhere."""
    rng = np.random.default_rng(n)
    F = rng.integers(0, 9, size=(n, n)).astype(float)
    D = rng.integers(0, 9, size=(n, n)).astype(float)
    Z = np.zeros((n,) * 6)
    for (i, j, k, p, q, r), vals in orbits:
        for mem, v in zip(_orbit_members(i, j, k, p, q, r), vals):
            Z[mem] = v
    da = O.DualAscent.from_arrays(F, D, np.zeros((n, n)), O.FULL, 0.0, np.zeros((n, n)),
                                  np.zeros((n,) * 4), Z)
    return da, Z


def test_f2_pool_worked_example():
    """Three members with slack 3, 1.5 and 6 give their 10.5 to the three
    with slack 0 (3.5 each) and drop to 0; an orbit with no zero slack, one
    with only zeros and the members outside every pooled orbit are
    untouched; a slack rounding left negative counts as zero."""
    n = 5
    a = (0, 1, 2, 0, 1, 2)
    b = (0, 1, 3, 4, 2, 0)
    c = (1, 2, 4, 3, 0, 1)
    d = (0, 3, 4, 1, 2, 3)
    orbits = [(a, [3.0, 0.0, 0.0, 1.5, 0.0, 6.0]),
              (b, [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]),
              (c, [0.0] * 6),
              (d, [2.0, -1e-15, 0.0, 0.0, 0.0, 0.0])]
    da, Z0 = _pool_state(n, orbits)
    da.pool()
    Z = da.export()[2]
    got = lambda o: [Z[mem] for mem in _orbit_members(*o)]
    assert got(a) == [0.0, 3.5, 3.5, 0.0, 3.5, 0.0]
    assert got(b) == [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    assert got(c) == [0.0] * 6
    assert got(d) == [0.0, -1e-15 + 0.4, 0.4, 0.4, 0.4, 0.4]
    touched = np.zeros_like(Z, dtype=bool)
    for o in (a, d):
        for mem in _orbit_members(*o):
            touched[mem] = True
    assert np.array_equal(Z[~touched], Z0[~touched])


@pytest.mark.parametrize("inst", [I.random_instance(6, 14), I.grid_instance(7, 2, 4, 0.4, 1, 9, 3)],
                         ids=lambda x: x.name)
def test_f2_pool_conserves_orbits_on_a_real_state(inst):
    """After a Z-LAP phase at t >= 1: every orbit's slack total is kept (to
    rounding), S_N members end at 0, S_B members all gain the same amount."""
    F, D, B = inst.arrays()
    n = inst.n
    da = O.DualAscent(F, D, B)
    da.run(3)
    da.sweep()
    da.zphase()
    Z0 = da.export()[2].copy()
    da.pool()
    Z1 = da.export()[2]
    pooled = 0
    for (i, j, k) in itertools.combinations(range(n), 3):
        for (p, q, r) in itertools.permutations(range(n), 3):
            mem = _orbit_members(i, j, k, p, q, r)
            v0 = np.array([Z0[x] for x in mem])
            v1 = np.array([Z1[x] for x in mem])
            assert abs(v1.sum() - v0.sum()) <= 1e-12 * max(1.0, np.abs(v0).sum())
            nb = int((v0 <= 0.0).sum())
            if nb in (0, 6):
                assert np.array_equal(v0, v1)
                continue
            pooled += 1
            assert np.all(v1[v0 > 0.0] == 0.0)
            gain = v1[v0 <= 0.0] - v0[v0 <= 0.0]
            assert np.allclose(gain, v0[v0 > 0.0].sum() / nb, rtol=1e-12, atol=0.0)
    assert pooled > 0


@pytest.mark.parametrize("inst", [I.random_instance(5, 3), I.grid_instance(6, 2, 3, 0.4, 1, 9, 4)],
                         ids=lambda x: x.name)
def test_f2_identity_every_phase(inst):
    """The pooling and the second Z-LAP solve keep the reformulation
    identity for every permutation, with reduced costs >= 0."""
    F, D, B = inst.arrays()
    n = F.shape[0]
    perms = [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
    da = O.DualAscent(F, D, B, two_phase=True)
    da.run(1)
    for _ in range(3):
        da.sweep()
        da.zphase()
        da.pool()
        _check_identity(da, F, D, B, perms)
        da.zphase()
        _check_identity(da, F, D, B, perms)
        da.yequal()
        da.yphase()
        da.xphase()
        _check_identity(da, F, D, B, perms)


@pytest.mark.parametrize("inst", [I.grid_n8(), I.random_instance(8, 3), I.dense_instance(9, 5)],
                         ids=lambda x: x.name)
def test_f2_bound_valid_monotone_and_at_least_f1(inst):
    """F2 bounds stay below the brute-force optimum and never fall; after 30
    iterations they are at least F1's on these instances (the paper's claim
    for two-phase variants), and on the 2x4 grid F2 proves the optimum."""
    F, D, B = inst.arrays()
    opt = brute_opt(F, D, B)
    f1 = O.DualAscent(F, D, B)
    f2 = O.DualAscent(F, D, B, two_phase=True)
    f1.run(30)
    f2.run(30)
    tr = f2.trace()
    assert np.all(np.diff(tr) >= 0.0)
    assert tr[-1] <= opt + 1e-9 * max(1.0, opt)
    assert f2.LB >= f1.LB - 1e-9 * max(1.0, opt)  # both may sit at the optimum, to rounding
    if inst.name.startswith("grid2x4"):
        assert f2.proven() and f2.UB == opt


def test_f2_refuses_half_and_tracking():
    inst = I.random_instance(5, 2)
    F, D, B = inst.arrays()
    with pytest.raises(ValueError):
        O.DualAscent(F, D, B, O.HALF, two_phase=True)
    da = O.DualAscent(F, D, B, two_phase=True)
    with pytest.raises(Exception):
        da.track()


# ---- Type 4 ascent with simulated annealing (Section 2.3, schedule of Section 5) ----

def test_splitmix64_published_outputs():
    """SplitMix64 seeded with 0: its first three outputs as published with
    the generator (Steele, Lea and Flood 2014); uniforms are the top 53 bits."""
    assert [O.splitmix64(0, c) for c in (1, 2, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                       0x06C45D188009454F]
    assert O.sa_uniform(0, 1) == (0xE220A8397B1DCDAF >> 11) / 2.0 ** 53
    u = [O.sa_uniform(7, c) for c in range(1, 20001)]
    assert min(u) >= 0.0 and max(u) < 1.0 and abs(np.mean(u) - 0.5) < 0.01


def test_sa_exp_matches_libm():
    import math
    xs = np.concatenate([np.linspace(-60.0, 0.0, 30001), -np.logspace(-12, 2.8, 2000)])
    for x in xs:
        e = math.exp(x)
        assert abs(O.sa_exp(x) - e) <= 4.5e-16 * e, x
    assert O.sa_exp(0.0) == 1.0 and O.sa_exp(-800.0) == 0.0


def _sa_state(inst, iters=3):
    F, D, B = inst.arrays()
    da = O.DualAscent(F, D, B)
    da.run(iters)
    return F, D, B, da


@pytest.mark.parametrize("inst", [I.random_instance(6, 21), I.grid_instance(6, 2, 3, 0.4, 1, 9, 5)],
                         ids=lambda x: x.name)
def test_type4_step_keeps_the_identity_and_moves_at_most_kappa_max(inst):
    """A taken Type 4 step (huge temperature) lowers LB by the amount it adds
    to the x slacks (each row i and column p uniformly), at most
    kappa_max * LB; every permutation's cost still equals LB + reduced costs
    and slacks stay >= 0.  A tiny temperature takes no step."""
    F, D, B, da = _sa_state(inst)
    n = inst.n
    perms = [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
    X0 = da.export()[0].copy()
    lb0 = da.LB
    da.set_annealing(1e30, kappa_max=0.25, seed=3)
    assert da.type4(5)
    X1 = da.export()[0]
    drop = lb0 - da.LB
    assert 0.0 < drop <= 0.25 * lb0 * (1 + 1e-12)
    inc = X1 - X0
    # row + column structure: inc[i,p] = a_i + b_p
    a = inc[:, 0] - inc[0, 0]
    b = inc[0, :]
    assert np.allclose(inc, a[:, None] + b[None, :], rtol=0, atol=1e-9 * lb0)
    assert abs(inc.trace() - drop) <= 1e-9 * lb0  # identity permutation meets each row/column once
    _check_identity(da, F, D, B, perms)
    F, D, B, db = _sa_state(inst)
    db.set_annealing(1e-300, seed=3)
    X0 = db.export()[0].copy()
    lb0 = db.LB
    assert not db.type4(5)
    assert db.LB == lb0 and np.array_equal(db.export()[0], X0)


@pytest.mark.parametrize("inst", [I.random_instance(8, 3), I.random_instance(9, 11)], ids=lambda x: x.name)
def test_annealed_ascent_bounds_stay_valid(inst):
    """With a temperature that takes nearly every step (each gives away up
    to a quarter of the bound), every iteration's bound stays <= the
    brute-force optimum and the final state keeps the identity."""
    F, D, B = inst.arrays()
    n = inst.n
    opt = brute_opt(F, D, B)
    da = O.DualAscent(F, D, B)
    da.run(2)
    da.set_annealing(10.0 * opt, seed=11)
    da.run(60)
    tr = da.trace()
    assert da.sa_accepted >= 0.5 * (da.t - 2) >= 4
    assert tr.max() <= opt + 1e-9 * max(1.0, opt)
    rng = np.random.default_rng(1)
    perms = [rng.permutation(n).astype(np.int32) for _ in range(200)]
    _check_identity(da, F, D, B, perms)


def test_annealing_schedule_and_refusals():
    """Section 5's schedule: at 4 % of the optimum a few steps are taken in
    300 iterations and the best bound is no worse than F1's; t0 <= 0 is F1
    exactly; bad parameters and tracking are refused."""
    inst = I.grid_instance(10, 2, 5, 0.4, 1, 9, 6)
    F, D, B = inst.arrays()
    f1 = O.DualAscent(F, D, B)
    f1.run(300)
    sa = O.DualAscent(F, D, B)
    sa.run(2)
    sa.set_annealing(0.04 * f1.UB, seed=1)
    sa.run(298)
    assert 1 <= sa.sa_accepted <= 50
    assert sa.trace().max() >= f1.LB
    off = O.DualAscent(F, D, B)
    off.set_annealing(0.0)
    off.run(40)
    assert np.array_equal(off.trace(), f1.trace()[:40])
    for bad in [dict(kappa_max=1.5), dict(cool=0.0), dict(period=0)]:
        with pytest.raises(ValueError):
            O.DualAscent(F, D, B).set_annealing(100.0, **bad)
    tr = O.DualAscent(F, D, B)
    tr.track()
    with pytest.raises(ValueError):
        tr.set_annealing(100.0)


# ---- slow variant S1 (Section 3.4): LAPs on the full costs every iteration ----

@pytest.mark.parametrize("inst", [I.random_instance(8, 3), I.grid_instance(9, 3, 3, 0.4, 1, 10, 2),
                                  I.random_instance(9, 11)], ids=lambda x: x.name)
def test_s1_bound_never_falls_and_stays_valid(inst):
    """Theorem 1 (fixed u): the S1 bounds, each recomputed from scratch on
    the full costs, never fall (to rounding) and stay below the brute-force
    optimum."""
    F, D, B = inst.arrays()
    opt = brute_opt(F, D, B)
    da = O.DualAscent(F, D, B, slow=True)
    da.run(30)
    tr = da.trace()
    assert np.all(np.diff(tr) >= -1e-9 * abs(tr[-1]))
    assert tr.max() <= opt + 1e-9 * max(1.0, opt)


def test_s1_state_is_the_s_form_of_its_multipliers():
    """After an S1 iteration the z level is -v for the tracked v (zero-sum
    over every orbit), the y multipliers are 0, and the bound of that
    iteration equals a fresh S-form start from v run for one iteration (the
    LAPs on b, C, -v) -- the left-hand side of Eq. ch4:proof:4."""
    inst = I.grid_instance(7, 2, 4, 0.4, 1, 9, 1)
    F, D, B = inst.arrays()
    n = inst.n
    da = O.DualAscent(F, D, B, slow=True)
    da.run(6)
    V, U = da.multipliers()
    assert not U.any()
    for (i, j, k) in itertools.combinations(range(n), 3):
        for (p, q, r) in [(0, 1, 2), (n - 1, 0, 3), (2, n - 2, 1)]:
            assert abs(sum(V[m] for m in _orbit_members(i, j, k, p, q, r))) <= 1e-9 * max(1.0, np.abs(V).max())
    # one more S1 iteration = sweep (v update), rebuild, LAPs
    da.run(1)
    V1, _ = da.multipliers()
    fresh = O.DualAscent.from_multipliers(F, D, B, O.FULL, V1, None)
    fresh.run(1)
    assert fresh.trace()[0] == da.trace()[-1]


@pytest.mark.parametrize("inst", [I.random_instance(5, 3), I.grid_instance(6, 2, 3, 0.4, 1, 9, 4)],
                         ids=lambda x: x.name)
def test_s1_identity_every_iteration(inst):
    F, D, B = inst.arrays()
    n = F.shape[0]
    perms = [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
    da = O.DualAscent(F, D, B, slow=True)
    for _ in range(5):
        da.run(1)
        _check_identity(da, F, D, B, perms)


def test_s1_refuses_other_variants():
    F, D, B = I.random_instance(5, 2).arrays()
    with pytest.raises(ValueError):
        O.DualAscent(F, D, B, O.HALF, slow=True)
    da = O.DualAscent(F, D, B, slow=True)
    with pytest.raises(ValueError):
        da.set_annealing(100.0)


@pytest.mark.parametrize("inst", [I.random_instance(8, 3), I.grid_instance(9, 3, 3, 0.4, 1, 10, 2)],
                         ids=lambda x: x.name)
def test_s2_pooling_moves_the_multipliers(inst):
    """S2 = S1 with F2's pooling, which in the S-form moves each pooled
    member's multiplier by (old slack - new slack): the multipliers stay
    zero-sum over every orbit, the state stays their S-form (z = -v after
    the next sweep), the identity holds, and the bounds never fall and stay
    below brute force."""
    F, D, B = inst.arrays()
    n = inst.n
    opt = brute_opt(F, D, B)
    da = O.DualAscent(F, D, B, two_phase=True, slow=True)
    da.run(12)
    tr = da.trace()
    assert np.all(np.diff(tr) >= -1e-9 * abs(tr[-1])) and tr.max() <= opt + 1e-9 * max(1.0, opt)
    V, U = da.multipliers()
    assert not U.any()
    scale = max(1.0, np.abs(V).max())
    for (i, j, k) in itertools.combinations(range(n), 3):
        for (p, q, r) in [(0, 1, 2), (n - 1, 0, 3), (2, n - 2, 1), (4, 3, 5)]:
            assert abs(sum(V[m] for m in _orbit_members(i, j, k, p, q, r))) <= 1e-9 * scale
    rng = np.random.default_rng(2)
    perms = [rng.permutation(n).astype(np.int32) for _ in range(200)]
    _check_identity(da, F, D, B, perms)
    # the pooling itself: old - new added to v, member by member
    da.sweep()
    V0, _ = da.multipliers()
    da.zphase()
    Z0 = da.export()[2].copy()
    da.pool()
    Z1 = da.export()[2]
    V1, _ = da.multipliers()
    assert np.allclose(V1 - V0, Z0 - Z1, rtol=0, atol=1e-12 * scale)


def test_z_tiles_accessor_matches_the_dense_export():
    """The tile accessor the full-size GPU parity test reads (rows k and
    columns r over the remaining indices, ascending) against the dense
    export of the same state, including a ragged tile choice."""
    from layout import dense_to_compact_z, tile_index

    inst = I.random_instance(7, 5)
    F, D, Bm = inst.arrays()
    da = O.DualAscent(F, D, Bm)
    da.run(3)
    _, _, Z = da.export()
    comp = dense_to_compact_z(7, Z)
    picks = [(0, 1, 0, 1), (6, 5, 6, 5), (3, 0, 2, 6), (2, 4, 5, 1)]
    got = da.z_tiles(picks)
    for a, (i, j, p, q) in enumerate(picks):
        assert np.array_equal(got[a], comp[tile_index(7, i, p, j, q)])
    with pytest.raises(ValueError):
        da.z_tiles([(1, 1, 0, 2)])
