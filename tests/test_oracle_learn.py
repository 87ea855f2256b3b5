"""Pins of the learned warm start's oracle (CPU only).

Each function of oracle/learn_oracle.py is checked against something other
than itself: hand-worked values, brute-force enumeration, a library routine
(torch's bfloat16 conversion), finite differences, closed forms of Adam, and
weak duality against the brute-force optimum.
"""
import itertools

import numpy as np
import pytest

from oracle import learn_oracle as L
from oracle import oracle as O
from paper_1710_03732_amd import instances as I


# ------------------------------------------------------------------ orbits --
@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_orbits_cover_every_z_variable_once(n):
    ids = np.arange(L.orbit_count(n))
    mem = L.members(n, ids)
    seen = set()
    for o in range(len(ids)):
        pairs = {(mem[o, 0, a], mem[o, 0, 3 + a]) for a in range(3)}
        for e in range(6):
            z = tuple(int(v) for v in mem[o, e])
            assert {(z[a], z[3 + a]) for a in range(3)} == pairs
            assert z not in seen
            seen.add(z)
    every = {(i, j, k, p, q, r)
             for (i, j, k) in itertools.permutations(range(n), 3)
             for (p, q, r) in itertools.permutations(range(n), 3)}
    assert seen == every


def test_orbit_id_order():
    """Facility triples lexicographically, then (p, q, r) in the order of
    itertools.permutations (which is the compressed index order)."""
    n = 5
    want = [(i, j, k, p, q, r) for (i, j, k) in itertools.combinations(range(n), 3)
            for (p, q, r) in itertools.permutations(range(n), 3)]
    got = [tuple(int(v) for v in row) for row in L.decode_orbits(n, np.arange(L.orbit_count(n)))]
    assert got == want


def test_members_hand_example():
    # n = 4, orbit 6: facilities (0,1,2), locations p=1, q=0, r=2
    assert L.decode_orbits(4, [6]).tolist() == [[0, 1, 2, 1, 0, 2]]
    assert L.members(4, [6])[0].tolist() == [
        [0, 1, 2, 1, 0, 2], [0, 2, 1, 1, 2, 0], [1, 0, 2, 0, 1, 2],
        [1, 2, 0, 0, 2, 1], [2, 0, 1, 2, 1, 0], [2, 1, 0, 2, 0, 1]]


# ---------------------------------------------------------------- features --
F4 = np.array([[1, 2, 0, 0], [4, 0, 3, 0], [0, 1, 0, 5], [2, 0, 0, 0]], dtype=float)
D4 = np.array([[0, 1, 2, 3], [1, 2, 4, 5], [2, 4, 0, 6], [3, 5, 6, 0]], dtype=float)
B4 = np.zeros((4, 4))
B4[0, 1] = 3.0


def test_features_hand_example():
    X = L.features(F4, D4, B4, [0, 6])
    # worked by hand: sF = 5, sD = 6, fbar = 17/12/5, dbar = 42/12/6
    want0 = [2 / 30, 4 / 30, 0, 0, 12 / 30, 4 / 30,
             0.6, 0.0, 0.4, 1 / 6, 1 / 3, 2 / 3,
             0.25, 0.25, 0.225, 0.25, 0.5, 0.5,
             0.0, 0.0, 0.0, 0.5,
             0.35, 0.0, 0.4 * 7 / 12, (1 / 6) * 17 / 60, (1 / 3) * 17 / 60, (2 / 3) * 17 / 60,
             0, 0, 0, 0]
    want6 = [1 / 15, 2 / 15, 0, 0, 0.2, 1 / 15,
             0.6, 0.0, 0.4, 1 / 6, 2 / 3, 1 / 3,
             0.25, 0.25, 0.225, 0.5, 0.25, 0.5,
             1 / 6, 0.0, 0.0, 0.5,
             0.35, 0.0, 0.4 * 7 / 12, (1 / 6) * 17 / 60, (2 / 3) * 17 / 60, (1 / 3) * 17 / 60,
             0, 0, 0, 0]
    np.testing.assert_allclose(X[0], want0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(X[1], want6, rtol=1e-12, atol=1e-15)


def test_features_follow_a_location_relabelling():
    inst = I.random_instance(6, 3, lo=0, hi=9)
    F, D, B = inst.arrays()
    rng = np.random.default_rng(1)
    sig = rng.permutation(6)                   # location l -> sig[l]
    inv = np.argsort(sig)
    D2 = D[np.ix_(inv, inv)]
    B2 = B[:, inv]
    ids = np.arange(L.orbit_count(6))
    o = L.decode_orbits(6, ids)
    X = L.features(F, D, B, ids)
    # the orbit (i,j,k, sig p, sig q, sig r) of the relabelled instance
    lookup = {tuple(int(v) for v in row): a for a, row in enumerate(o)}
    ids2 = [lookup[(r[0], r[1], r[2], sig[r[3]], sig[r[4]], sig[r[5]])] for r in o]
    X2 = L.features(F, D2, B2, ids2)
    np.testing.assert_allclose(X2, X, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- bfloat16 --
def test_bf16_rounding_hand_values():
    e = 2.0 ** -8
    vals = [1.0, 1 + e, 1 + 3 * e, 1 + e + 2.0 ** -20, -(1 + 3 * e), 0.0, 3.0, 2.0 ** -130]
    want = [1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -(1 + 4 * e), 0.0, 3.0, 2.0 ** -130]
    np.testing.assert_array_equal(L.bf16(vals), want)


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(2).standard_normal(20000) * np.exp(np.random.default_rng(3).uniform(-30, 30, 20000))
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(L.bf16(x), ref)


# -------------------------------------------------------------- perceptron --
def _hand_params():
    W1 = np.zeros((256, 32))
    W1[0, 0] = 1.0
    W1[1, 1] = 1.0
    W2 = np.zeros((256, 256))
    W2[0, 0] = 3.0
    W3 = np.zeros((6, 256))
    W3[:, 0] = np.arange(6)
    return L.Params(W1, np.zeros(256), W2, np.zeros(256), W3, np.full(6, 0.5))


@pytest.mark.parametrize("rounding", [False, True])
def test_forward_hand_network(rounding):
    X = np.zeros((1, 32))
    X[0, 0], X[0, 1] = 1.0, -2.0
    y, c = L.forward(_hand_params(), X, rounding)
    # h1 = relu(1, -2) = (1, 0); h2_0 = 3; y_e = 3 e + 0.5
    np.testing.assert_array_equal(c["h1"][0, :2], [1.0, 0.0])
    np.testing.assert_array_equal(y[0], [0.5, 3.5, 6.5, 9.5, 12.5, 15.5])
    np.testing.assert_array_equal(L.project(y)[0], [-7.5, -4.5, -1.5, 1.5, 4.5, 7.5])


def test_projection():
    y = np.random.default_rng(4).standard_normal((50, 6))
    p = L.project(y)
    assert np.abs(p.sum(1)).max() < 1e-14
    np.testing.assert_allclose(L.project(p), p, atol=1e-15)


def _small_params(rng, w=8):
    return L.Params(rng.standard_normal((w, 32)) * 0.5, rng.standard_normal(w) * 0.1,
                    rng.standard_normal((w, w)) * 0.5, rng.standard_normal(w) * 0.1,
                    rng.standard_normal((6, w)) * 0.5, rng.standard_normal(6) * 0.1)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(5)
    P = _small_params(rng)
    X = rng.standard_normal((7, 32))
    T = L.project(rng.standard_normal((7, 6)))
    G = L.gradients(P, X, T, rounding=False)
    h = 1e-6
    for name in L.Params.NAMES:
        A = getattr(P, name)
        num = np.zeros_like(A)
        for idx in np.ndindex(A.shape):
            keep = A[idx]
            A[idx] = keep + h
            lp = L.loss(L.forward(P, X, False)[0], T)
            A[idx] = keep - h
            lm = L.loss(L.forward(P, X, False)[0], T)
            A[idx] = keep
            num[idx] = (lp - lm) / (2 * h)
        err = np.abs(G[name] - num).max() / max(1e-12, np.abs(num).max())
        assert err <= 1e-6, (name, err)


def test_rounded_gradients_close_to_exact():
    """The bfloat16 roundings perturb each term by about 2^-8 relative (more
    after cancellation over many samples); a dropped term or a transposed
    operand moves the gradient by order one."""
    rng = np.random.default_rng(6)
    P = L.Params(rng.standard_normal((256, 32)) * 0.2, rng.standard_normal(256) * 0.1,
                 rng.standard_normal((256, 256)) * 0.06, rng.standard_normal(256) * 0.1,
                 rng.standard_normal((6, 256)) * 0.06, rng.standard_normal(6) * 0.1)
    for N, tol in ((1, 3e-2), (64, 1e-1)):
        X = rng.standard_normal((N, 32))
        T = L.project(rng.standard_normal((N, 6)))
        Ge = L.gradients(P, X, T, rounding=False)
        Gr = L.gradients(P, X, T, rounding=True)
        for name in L.Params.NAMES:
            rel = np.linalg.norm(Gr[name] - Ge[name]) / np.linalg.norm(Ge[name])
            assert rel < tol, (N, name, rel)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2
    at every step, so each step moves w by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 8):
        w2, m, v = L.adam_step(w, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(w2 - w, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
        w = w2


# -------------------------------------------------------------- warm start --
@pytest.mark.parametrize("inst", [I.random_instance(7, 21), I.dense_instance(7, 22), I.grid_instance(8, 2, 4, 0.4, 1, 9, 23)],
                         ids=lambda x: x.name)
def test_warm_start_from_any_outputs_is_a_valid_bound(inst):
    F, D, B = inst.arrays()
    n = inst.n
    opt, _ = O.bruteforce(F, D, B)
    rng = np.random.default_rng(7)
    _, _, scale = L.scales(F, D)
    for spread in (0.1, 1.0, 10.0):
        y = (rng.standard_normal((L.orbit_count(n), 6)) * spread).astype(np.float32)
        V = L.multipliers_from_outputs(n, y, scale)
        mem = L.members(n, np.arange(L.orbit_count(n)))
        sums = V[tuple(mem.reshape(-1, 6).T)].reshape(-1, 6).sum(1)
        assert np.abs(sums).max() <= 1e-12 * max(1.0, np.abs(V).max())
        w = O.DualAscent.from_multipliers(F, D, B, O.FULL, V, None)
        w.run(6)
        assert np.all(w.trace() <= opt + 1e-9 * abs(opt))


def test_targets_round_trip():
    """Outputs placed as multipliers and gathered back as targets give the
    projected outputs."""
    n = 6
    F, D, B = I.random_instance(n, 8).arrays()
    _, _, scale = L.scales(F, D)
    y = np.random.default_rng(9).standard_normal((L.orbit_count(n), 6)).astype(np.float32)
    V = L.multipliers_from_outputs(n, y, scale)
    ids = np.random.default_rng(10).choice(L.orbit_count(n), 300, replace=False)
    t = L.targets(V, ids, scale)
    np.testing.assert_allclose(t, L.project(y[ids].astype(np.float64)), rtol=1e-6, atol=1e-6)


def test_tracked_targets_are_zero_sum():
    inst = I.grid_n8()
    F, D, B = inst.arrays()
    da = O.DualAscent(F, D, B)
    da.track()
    da.run(20)
    V, _ = da.multipliers()
    _, _, scale = L.scales(F, D)
    t = L.targets(V, np.arange(L.orbit_count(8)), scale).astype(np.float64)
    assert np.abs(t.sum(1)).max() <= 1e-5 * max(1.0, np.abs(t).max())
    assert np.abs(t).max() > 0


def test_s_form_start_keeps_the_reformulation_identity():
    """After a start from zero-sum multipliers (z costs -v) the reformulation
    identity cost(perm) = LB + sum of reduced costs holds for every
    permutation, at t = 0 (each orbit a permutation selects is selected whole,
    so its -v sum vanishes) and after further iterations."""
    inst = I.random_instance(6, 50, lo=-3, hi=8)
    F, D, B = inst.arrays()
    n = 6
    _, _, scale = L.scales(F, D)
    y = np.random.default_rng(51).standard_normal((L.orbit_count(n), 6)).astype(np.float32)
    w = O.DualAscent.from_multipliers(F, D, B, O.FULL, L.multipliers_from_outputs(n, y, scale), None)
    perms = [np.array(p, dtype=np.int32) for p in itertools.islice(itertools.permutations(range(n)), 0, 720, 37)]
    for steps in (0, 1, 4):
        if steps:
            w.run(steps)
        for p in perms:
            cost = O.qap_cost(F, D, B, p)
            assert abs(w.identity(p) - cost) <= 1e-9 * max(1.0, abs(cost)) * 100
