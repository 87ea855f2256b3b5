"""GPU parity of multiplier tracking, the S-form restart and the learned warm
start, through the C ABI.

Bitwise against the oracle: tracked multipliers, the S-form restart and the
z writer (fed the oracle's outputs), the targets gather.  Within tolerance:
features (float32 vs float64), the perceptron's outputs and gradients entry
by entry (the oracle in float64 on identically bf16-rounded operands, with
the per-entry bounds of bf16_bounds: every entry within the worst case of
float32 accumulation plus flipped bf16 rounding decisions, and almost every
entry of each output column within the bound with no flipped decision),
and warm-start bounds.  Validity: every warm-started bound stays below the
brute-force optimum.
"""
import numpy as np
import pytest

from bf16_bounds import assert_within, forward_bounds, gradient_bounds
from layout import dense_to_compact_y, dense_to_compact_z
from oracle import learn_oracle as L
from oracle import oracle as O
from paper_1710_03732_amd import binding as B
from paper_1710_03732_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((256, 32)) * 0.25 * scale, "b1": rng.standard_normal(256) * 0.05,
            "W2": rng.standard_normal((256, 256)) * 0.09 * scale, "b2": rng.standard_normal(256) * 0.05,
            "W3": rng.standard_normal((6, 256)) * 0.09 * scale, "b3": rng.standard_normal(6) * 0.05}


def _oracle_params(p):
    return L.Params(p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])


# GPU features are float32 (within 2e-6 relative of the oracle's) before
# their bf16 rounding; a rounding decision of an input can flip
FEATURE_REL = 4e-6


def _check_outputs(y, yo, P, X, name, feature_rel=0.0, frac=0.01):
    """GPU outputs y against the oracle's yo, entry by entry (and their
    zero-sum projections)."""
    f = forward_bounds(P, X, feature_rel=feature_rel)
    nf = forward_bounds(P, X, feature_rel=feature_rel, flips=False)
    assert np.allclose(f["y"], yo, rtol=1e-12, atol=1e-300), "bounds taken on another forward pass"
    # the fraction test needs enough rows for one flipped decision to be rare
    few = len(yo) < 200
    assert_within(y, yo, f["dy"], name, noflip=None if few else nf["dy"], axis=1, frac=frac)
    proj_w = f["dy"] + f["dy"].mean(axis=1, keepdims=True)
    proj_n = nf["dy"] + nf["dy"].mean(axis=1, keepdims=True)
    assert_within(L.project(np.asarray(y, np.float64)), L.project(yo), proj_w, name + " projected",
                  noflip=None if few else proj_n, axis=1, frac=frac)


def _compact_v(n, V):
    return dense_to_compact_z(n, V).reshape(-1)


def _state_equal(gpu, cpu):
    hdr, x, y, z = gpu.export_state()
    X, Y, Z = cpu.export()
    n = cpu.n
    assert hdr.t == cpu.t
    assert hdr.lb == cpu.LB, (hdr.lb, cpu.LB)
    assert np.array_equal(x, X.reshape(-1))
    assert np.array_equal(y, dense_to_compact_y(n, Y))
    assert np.array_equal(z.reshape(-1, n - 2, n - 2), dense_to_compact_z(n, Z))


INSTS = [I.random_instance(7, 80), I.grid_n8(), I.dense_instance(8, 81), I.random_instance(6, 82, lo=-3, hi=9)]


@pytest.mark.parametrize("inst", INSTS, ids=lambda x: x.name)
def test_tracked_multipliers_bitwise(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    g = B.DualAscent(F, D, Bm)
    c = O.DualAscent(F, D, Bm)
    g.track()
    c.track()
    for step in (1, 3, 5):
        g.run(step)
        c.run(step)
        v, u = g.multipliers()
        V, U = c.multipliers()
        assert np.array_equal(v, _compact_v(n, V))
        assert np.array_equal(u, dense_to_compact_y(n, U))
        _state_equal(g, c)


@pytest.mark.parametrize("inst", INSTS[:3], ids=lambda x: x.name)
def test_s_form_restart_bitwise(inst):
    """Restart from the oracle's tracked multipliers: same arrays and the same
    trajectory as the oracle's restart."""
    F, D, Bm = inst.arrays()
    n = inst.n
    c = O.DualAscent(F, D, Bm)
    c.track()
    c.run(12)
    V, U = c.multipliers()
    g = B.DualAscent(F, D, Bm)
    g.run(2)
    g.set_multipliers(_compact_v(n, V), dense_to_compact_y(n, U))
    w = O.DualAscent.from_multipliers(F, D, Bm, O.FULL, V, U)
    _state_equal(g, w)
    g.run(1)
    w.run(1)
    assert g.trace()[0] >= c.trace()[-1] - 1e-9 * abs(c.trace()[-1])
    for _ in range(4):
        g.run(1)
        w.run(1)
        _state_equal(g, w)
    assert np.array_equal(g.trace(), w.trace())


def test_set_multipliers_rejects_non_zero_sum():
    F, D, Bm = I.random_instance(6, 83).arrays()
    g = B.DualAscent(F, D, Bm)
    v = np.zeros(g.T * g.m * g.m)
    v[5] = 1.0
    with pytest.raises(B.QapError) as e:
        g.set_multipliers(v, None)
    assert e.value.code == -1
    u = np.zeros(g.T)
    u[3] = 2.0
    with pytest.raises(B.QapError):
        g.set_multipliers(None, u)


@pytest.mark.parametrize("inst", [I.random_instance(9, 84, lo=-4, hi=20), I.grid_n8(), I.dense_n14()],
                         ids=lambda x: x.name)
def test_orbit_features_and_scale(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    g = B.DualAscent(F, D, Bm)
    cnt = B.orbit_count(n)
    assert cnt == L.orbit_count(n)
    ids = np.unique(np.concatenate([np.random.default_rng(85).integers(0, cnt, 3000), [0, cnt - 1]]))
    x = g.orbit_features(torch.tensor(ids, dtype=torch.int64, device="cuda")).cpu().numpy()
    X = L.features(F, D, Bm, ids)
    np.testing.assert_allclose(x, X, rtol=2e-6, atol=1e-7)
    assert g.multiplier_scale() == L.scales(F, D)[2]


def test_orbit_targets_bitwise():
    inst = I.dense_instance(8, 86)
    F, D, Bm = inst.arrays()
    g = B.DualAscent(F, D, Bm)
    c = O.DualAscent(F, D, Bm)
    g.track()
    c.track()
    g.run(9)
    c.run(9)
    V, _ = c.multipliers()
    scale = L.scales(F, D)[2]
    ids = np.random.default_rng(87).permutation(L.orbit_count(8))[:5000]
    t = g.orbit_targets(torch.tensor(ids, dtype=torch.int64, device="cuda"), scale).cpu().numpy()
    assert np.array_equal(t, L.targets(V, ids, scale))


@pytest.mark.parametrize("inst", [I.random_instance(7, 88), I.grid_n8(), I.dense_instance(9, 89)],
                         ids=lambda x: x.name)
def test_warm_start_writer_bitwise(inst):
    """Per-orbit outputs from the shared seeded generator: the GPU's S-form
    restart equals the oracle's, array for array, and so does the run."""
    F, D, Bm = inst.arrays()
    n = inst.n
    y = (np.random.default_rng(90).standard_normal((L.orbit_count(n), 6)) * 0.3).astype(np.float32)
    scale = L.scales(F, D)[2]
    g = B.DualAscent(F, D, Bm)
    g.run(3)
    g.warm_start_outputs(torch.tensor(y, device="cuda"), scale)
    w = O.DualAscent.from_multipliers(F, D, Bm, O.FULL, L.multipliers_from_outputs(n, y, scale), None)
    _state_equal(g, w)
    g.run(5)
    w.run(5)
    _state_equal(g, w)
    assert np.array_equal(g.trace(), w.trace())
    opt, _ = O.bruteforce(F, D, Bm)
    assert np.all(g.trace() <= opt + 1e-9 * abs(opt))


def test_mlp_forward_matches_oracle():
    p = _params(91)
    mlp = B.Mlp(p, max_batch=2048)
    x = np.random.default_rng(92).standard_normal((1500, 32)).astype(np.float32)
    y = mlp.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    P = _oracle_params(p)
    yo, _ = L.forward(P, x.astype(np.float64), rounding=True)
    _check_outputs(y, yo, P, x, "forward")


@pytest.mark.parametrize("inst", [I.grid_n8(), I.dense_instance(10, 93)], ids=lambda x: x.name)
def test_fused_orbit_outputs_match_oracle(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    p = _params(94)
    mlp = B.Mlp(p, max_batch=4096)
    g = B.DualAscent(F, D, Bm)
    y = g.orbit_outputs(mlp).cpu().numpy()
    X = L.features(F, D, Bm, np.arange(L.orbit_count(n)))
    P = _oracle_params(p)
    yo, _ = L.forward(P, X, rounding=True)
    _check_outputs(y, yo, P, X, "fused outputs", feature_rel=FEATURE_REL, frac=0.05)
    # the training path's GEMM forward on the GPU's own features: both
    # sides round the same float32 features, each is within its bound of
    # the oracle, so they are within twice the bound of each other
    ids = torch.arange(0, min(4096, L.orbit_count(n)), dtype=torch.int64, device="cuda")
    yg = mlp.forward(g.orbit_features(ids)).cpu().numpy()
    k = len(yg)
    f = forward_bounds(P, X[:k], feature_rel=FEATURE_REL)
    assert_within(yg, y[:k], 2 * f["dy"], "GEMM forward vs fused")


def test_mlp_gradients_match_oracle():
    p = _params(95)
    mlp = B.Mlp(p, max_batch=1024)
    rng = np.random.default_rng(96)
    x = rng.standard_normal((700, 32)).astype(np.float32)
    t = L.project(rng.standard_normal((700, 6)) * 0.5).astype(np.float32)
    g, loss = mlp.gradients(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"))
    P = _oracle_params(p)
    G = L.gradients(P, x.astype(np.float64), t.astype(np.float64), rounding=True)
    yo, _ = L.forward(P, x.astype(np.float64), rounding=True)
    assert abs(loss - L.loss(yo, t)) <= 1e-4 * L.loss(yo, t)
    gg = B.unpack_mlp_params(g)
    worst = gradient_bounds(P, x, t)
    nf = gradient_bounds(P, x, t, flips=False)
    for name in L.Params.NAMES:
        assert_within(gg[name], G[name], worst[name], "gradient " + name, noflip=nf[name], frac=0.05)


def test_adam_step_closed_form():
    """First Adam step: w moves by -lr g / (|g| + eps) with g the gradient of
    the same batch (bias-corrected moments are g and g^2)."""
    p = _params(97)
    mlp = B.Mlp(p, max_batch=512)
    rng = np.random.default_rng(98)
    x = torch.tensor(rng.standard_normal((300, 32)).astype(np.float32), device="cuda")
    t = torch.tensor(L.project(rng.standard_normal((300, 6))).astype(np.float32), device="cuda")
    w0 = mlp.params()
    g, _ = mlp.gradients(x, t)
    lr = 1e-3
    mlp.train_step(x, t, lr=lr)
    w1 = mlp.params()
    want = -lr * g.astype(np.float64) / (np.abs(g.astype(np.float64)) + 1e-8)
    np.testing.assert_allclose(w1.astype(np.float64) - w0, want, rtol=1e-3, atol=2e-9)


def test_training_reduces_loss_on_tracked_targets():
    inst = I.dense_instance(9, 99)
    F, D, Bm = inst.arrays()
    g = B.DualAscent(F, D, Bm)
    g.track()
    g.run(30)
    scale = g.multiplier_scale()
    ids = torch.randperm(B.orbit_count(9), generator=torch.Generator().manual_seed(100))[:8192].to("cuda")
    x = g.orbit_features(ids)
    t = g.orbit_targets(ids, scale)
    mlp = B.Mlp(_params(101, scale=0.5), max_batch=8192)
    first = mlp.train_step(x, t, lr=1e-3)
    for _ in range(150):
        last = mlp.train_step(x, t, lr=1e-3)
    assert last < 0.5 * first, (first, last)


@pytest.mark.parametrize("inst", [I.grid_n8(), I.dense_instance(8, 102), I.random_instance(8, 103, lo=-5, hi=9)],
                         ids=lambda x: x.name)
def test_learned_warm_start_is_valid_and_matches_oracle(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    opt, _ = O.bruteforce(F, D, Bm)
    p = _params(104)
    mlp = B.Mlp(p, max_batch=1024)
    g = B.DualAscent(F, D, Bm)
    st = g.warm_start(mlp)
    assert st["orbits"] == L.orbit_count(n)
    g.run(10)
    tr = g.trace()
    assert np.all(tr <= opt + 1e-9 * abs(opt))
    # the oracle's warm start from its own forward pass
    X = L.features(F, D, Bm, np.arange(L.orbit_count(n)))
    yo, _ = L.forward(_oracle_params(p), X, rounding=True)
    w = O.DualAscent.from_multipliers(F, D, Bm, O.FULL,
                                      L.multipliers_from_outputs(n, yo.astype(np.float32), L.scales(F, D)[2]), None)
    w.run(1)
    assert abs(tr[0] - w.trace()[0]) <= 1e-3 * max(1.0, abs(w.trace()[0]))


@pytest.mark.parametrize("idx", [66, 67], ids=["fam66_grid_n20", "fam67_dense_n20"])
def test_trained_warm_start_beats_cold_on_heldout(idx):
    """The committed weights (trained on idx < 64) on held-out instances:
    the warm start reaches the bound of 100 cold iterations in fewer
    iterations, and every warm bound stays below the incumbent."""
    from paper_1710_03732_amd import train_warm

    inst = I.learned_family(idx)
    F, D, Bm = inst.arrays()
    mlp = B.Mlp(train_warm.load_weights(), max_batch=256)
    cold = B.DualAscent(F, D, Bm)
    rc = cold.run(100)
    warm = B.DualAscent(F, D, Bm)
    warm.warm_start(mlp)
    rw = warm.run(100)
    tr = np.maximum.accumulate(warm.trace())
    ub = min(rc["ub"], rw["ub"])
    assert np.all(warm.trace() <= ub + 1e-9 * ub)
    hit = np.nonzero(tr >= rc["lb"])[0]
    assert len(hit) and hit[0] + 1 <= 80, (hit[:1], rc["lb"], tr[-1])


@pytest.mark.parametrize("n", [3, 4])
def test_warm_start_smallest_sizes(n):
    """One facility triple (n = 3, six orbits, 1x1 Z-LAPs): writer and
    inference still agree with the oracle and the bound stays valid."""
    inst = I.random_instance(n, 30 + n, lo=0, hi=9)
    F, D, Bm = inst.arrays()
    opt, _ = O.bruteforce(F, D, Bm)
    y = (np.random.default_rng(n).standard_normal((L.orbit_count(n), 6))).astype(np.float32)
    scale = L.scales(F, D)[2]
    g = B.DualAscent(F, D, Bm)
    g.warm_start_outputs(torch.tensor(y, device="cuda"), scale)
    w = O.DualAscent.from_multipliers(F, D, Bm, O.FULL, L.multipliers_from_outputs(n, y, scale), None)
    _state_equal(g, w)
    g.run(4)
    w.run(4)
    assert np.array_equal(g.trace(), w.trace())
    assert np.all(g.trace() <= opt + 1e-9 * abs(opt))
    mlp = B.Mlp(_params(105), max_batch=64)
    yo = g.orbit_outputs(mlp).cpu().numpy()
    X = L.features(F, D, Bm, np.arange(L.orbit_count(n)))
    P = _oracle_params(_params(105))
    ref, _ = L.forward(P, X, True)
    _check_outputs(yo, ref, P, X, "fused outputs", feature_rel=FEATURE_REL, frac=0.05)


def test_warm_start_gain_scales_the_multipliers():
    """qap_warm_start with a gain equals the writer fed the same outputs at
    scale * gain (bitwise), and any gain keeps the bound valid."""
    inst = I.dense_instance(8, 106)
    F, D, Bm = inst.arrays()
    opt, _ = O.bruteforce(F, D, Bm)
    mlp = B.Mlp(_params(107), max_batch=64)
    a = B.DualAscent(F, D, Bm)
    st = a.warm_start(mlp, gain=2.5)
    assert st["gain"] == 2.5 and st["scale"] == a.multiplier_scale() * 2.5
    b = B.DualAscent(F, D, Bm)
    b.warm_start_outputs(b.orbit_outputs(mlp), b.multiplier_scale() * 2.5)
    for h in (a, b):
        h.run(6)
    assert np.array_equal(a.trace(), b.trace())
    assert np.all(a.trace() <= opt + 1e-9 * abs(opt))
    with pytest.raises(B.QapError):
        a.warm_start(mlp, gain=0.0)


def test_later_allocations_through_a_caller_allocator():
    """qap_set_allocator: tracking arrays and the learned calls' buffers come
    from torch's caching allocator; results equal the hipMalloc handle's."""
    F, D, Bm = I.dense_instance(8, 108).arrays()
    seen = []

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes)
        seen.append(nbytes)
        return p

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    a = B.DualAscent(F, D, Bm)
    a.set_allocator(alloc, free)
    a.track()
    a.run(4)
    b = B.DualAscent(F, D, Bm)
    b.track()
    b.run(4)
    va, ua = a.multipliers()
    vb, ub = b.multipliers()
    assert np.array_equal(va, vb) and np.array_equal(ua, ub)
    mlp = B.Mlp(_params(109), max_batch=64)
    a.track(False)
    a.warm_start(mlp)
    b.track(False)
    b.warm_start(mlp)
    a.run(3)
    b.run(3)
    assert np.array_equal(a.trace(), b.trace())
    assert len(seen) >= 3  # two tracking arrays, then the warm start's buffers
    with pytest.raises(B.QapError):
        a.track()
        a.set_allocator(None)  # refused while tracking arrays are live
    a.track(False)
    a.set_allocator(None)
