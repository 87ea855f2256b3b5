"""The element-wise bf16 error bounds used by the GPU perceptron tests hold
for a float32 emulation of the GPU's arithmetic (same bf16 roundings,
float32 accumulation in another order) and reject a planted one-weight
mistake that a norm ratio of 1e-3 lets through."""
import numpy as np

from bf16_bounds import assert_within, forward_bounds, gradient_bounds
from oracle import learn_oracle as L


def _params(seed):
    rng = np.random.default_rng(seed)
    return L.Params(rng.standard_normal((256, 32)) * 0.25, rng.standard_normal(256) * 0.05,
                    rng.standard_normal((256, 256)) * 0.09, rng.standard_normal(256) * 0.05,
                    rng.standard_normal((6, 256)) * 0.09, rng.standard_normal(6) * 0.05)


def _forward_f32(P, X):
    """bf16 operands, float32 accumulation in reversed column order."""
    r = L.bf16
    f32 = np.float32

    def mm(a, w):  # a [N,K] @ w.T [K,M], summed from the last k down in float32
        a = a.astype(f32)
        w = w.astype(f32)
        acc = np.zeros((a.shape[0], w.shape[0]), f32)
        for k in range(a.shape[1] - 1, -1, -1):
            acc = (acc + a[:, k:k + 1] * w[:, k][None, :]).astype(f32)
        return acc

    x = r(X)
    h1 = np.maximum(mm(x, r(P.W1)) + P.b1.astype(f32), 0).astype(f32)
    h2 = np.maximum(mm(r(h1), r(P.W2)) + P.b2.astype(f32), 0).astype(f32)
    return (mm(r(h2), r(P.W3)) + P.b3.astype(f32)).astype(np.float64)


def test_float32_emulation_within_forward_bounds():
    P = _params(1)
    X = np.random.default_rng(2).standard_normal((400, 32)).astype(np.float32)
    f = forward_bounds(P, X)
    nf = forward_bounds(P, X, flips=False)
    y = _forward_f32(P, X)
    worst = assert_within(y, f["y"], f["dy"], "y", noflip=nf["dy"], axis=1)
    assert worst < 1.0


def test_planted_weight_error_is_caught_elementwise():
    """One wrong W3 entry: the Frobenius ratio stays far under 1e-3 while
    the output column it feeds falls outside the no-flip bound."""
    P = _params(3)
    X = np.random.default_rng(4).standard_normal((400, 32)).astype(np.float32)
    f = forward_bounds(P, X)
    nf = forward_bounds(P, X, flips=False)
    Q = L.Params(P.W1, P.b1, P.W2, P.b2, P.W3.copy(), P.b3)
    Q.W3[2, 17] += 0.003
    y = _forward_f32(Q, X)
    rel = np.linalg.norm(y - f["y"]) / np.linalg.norm(f["y"])
    assert rel < 1e-3
    try:
        assert_within(y, f["y"], f["dy"], "y", noflip=nf["dy"], axis=1)
    except AssertionError:
        return
    raise AssertionError("planted error not detected")


def test_gradient_bounds_shapes_and_planted_error():
    """The gradient bounds have the gradients' shapes, the worst case covers
    the no-flip case, and an entry moved far beyond its bound is flagged."""
    P = _params(5)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((300, 32)).astype(np.float32)
    T = L.project(rng.standard_normal((300, 6)) * 0.5).astype(np.float32)
    bnd = gradient_bounds(P, X, T)
    nf = gradient_bounds(P, X, T, flips=False)
    G = L.gradients(P, X.astype(np.float64), T.astype(np.float64), rounding=True)
    for name in L.Params.NAMES:
        assert bnd[name].shape == np.shape(G[name])
        assert np.all(bnd[name] >= nf[name]) and np.all(nf[name] >= 0)
    # a perturbation of one gradient entry far beyond the bound is flagged
    bad = G["W2"].copy()
    bad[5, 9] += 100 * bnd["W2"][5, 9] + 1e-6
    try:
        assert_within(bad, G["W2"], bnd["W2"], "W2")
    except AssertionError:
        return
    raise AssertionError("planted gradient error not detected")
