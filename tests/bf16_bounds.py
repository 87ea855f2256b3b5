"""Element-wise error bounds for the perceptron's bf16 products.

The GPU rounds every product operand to bfloat16 (as the oracle does with
rounding on) but accumulates in float32 in its own order, so the two sides
differ by (a) float32 accumulation error and (b) bfloat16 rounding
decisions that the accumulation error can flip.  These helpers propagate
worst-case bounds for both, entry by entry, through the forward and
backward passes, from the oracle's own activations:

* a float32 sum of K products (plus a bias) is within gamma(K) times the
  sum of the magnitudes of its terms, gamma(K) = (K + 2) 2^-24;
* rounding to bfloat16 moves a value by at most one unit in the last place
  of its larger neighbour, at most 2^-7 of its magnitude, so two inputs
  that differ by d round to values that differ by at most
  d + 2^-7 (|value| + d);
* a ReLU mask (or the mask of the backward pass) can differ only where the
  pre-activation is within its own error bound of zero; there the whole
  term is allowed to differ.

Test helpers only: no part of the method is computed here.
"""
from __future__ import annotations

import numpy as np

U7 = 2.0 ** -7


def gamma(k: int) -> float:
    return (k + 2) * 2.0 ** -24


def _env(a, b_t):
    """sum_k |a_ik| |b_jk| (the magnitude envelope of a @ b_t.T)."""
    return np.abs(a) @ np.abs(b_t).T


def _round_gap(v, d, flips: bool = True):
    """Bound on |bf16(v + e) - bf16(v)| for |e| <= d; without flips (both
    sides took the same rounding decision) the rounded values are equal."""
    if not flips:
        return np.zeros_like(np.asarray(v, np.float64))
    return d + U7 * (np.abs(v) + d)


def forward_bounds(P, X, feature_rel: float = 0.0, flips: bool = True):
    """Per-entry bounds on |y_gpu - y_oracle| and on the hidden activations,
    for the oracle's rounded forward pass of parameters P on inputs X.
    `feature_rel` is the relative error of the inputs before their rounding
    (0 when both sides round the same float32 inputs).  With flips=False
    the bound assumes every bfloat16 rounding decision agrees (what almost
    every entry sees): then only the last product's accumulation differs."""
    from oracle import learn_oracle as L

    r = L.bf16
    x = r(X)
    W1, W2, W3 = r(P.W1), r(P.W2), r(P.W3)
    dx = (_round_gap(x, feature_rel * np.abs(np.asarray(X, np.float64)), flips) if feature_rel
          else np.zeros_like(x))
    a1 = x @ W1.T + P.b1
    e1 = _env(x, W1) + np.abs(P.b1)
    da1 = gamma(W1.shape[1]) * e1 + np.abs(dx) @ np.abs(W1).T
    h1 = np.maximum(a1, 0.0)
    dh1 = _round_gap(h1, da1, flips)
    h1r = r(h1)
    a2 = h1r @ W2.T + P.b2
    e2 = _env(h1r, W2) + np.abs(P.b2)
    da2 = gamma(W2.shape[1]) * e2 + dh1 @ np.abs(W2).T
    h2 = np.maximum(a2, 0.0)
    dh2 = _round_gap(h2, da2, flips)
    h2r = r(h2)
    y = h2r @ W3.T + P.b3
    e3 = _env(h2r, W3) + np.abs(P.b3)
    dy = gamma(W3.shape[1]) * e3 + dh2 @ np.abs(W3).T
    return {"y": y, "dy": dy, "x": x, "dx": dx, "a1": a1, "da1": da1, "h1": h1, "h1r": h1r, "dh1": dh1,
            "a2": a2, "da2": da2, "h2": h2, "h2r": h2r, "dh2": dh2, "W1": W1, "W2": W2, "W3": W3}


def gradient_bounds(P, X, T, flips: bool = True):
    """Per-entry bounds on the six gradient tensors of the projected MSE
    (the oracle's rounded backward pass), given the forward bounds; with
    flips=False every rounding decision and every ReLU mask is taken to
    agree."""
    from oracle.learn_oracle import bf16

    f = forward_bounds(P, X, flips=flips)
    N = f["y"].shape[0]
    y, dy = f["y"], f["dy"]
    Tm = np.asarray(T, np.float64)
    proj = y - y.mean(axis=1, keepdims=True)
    g = 2.0 * (proj - Tm) / (6.0 * N)
    d3 = g - g.mean(axis=1, keepdims=True)
    dproj = dy + dy.mean(axis=1, keepdims=True)
    dg = 2.0 / (6.0 * N) * dproj + gamma(6) * np.abs(g)
    dd3 = dg + dg.mean(axis=1, keepdims=True) + gamma(6) * np.abs(d3)
    d3r = bf16(d3)
    dd3r = _round_gap(d3, dd3, flips)
    h2r, dh2, h1r, dh1 = f["h2r"], f["dh2"], f["h1r"], f["dh1"]
    W2, W3 = f["W2"], f["W3"]
    out = {}
    out["W3"] = (dd3r.T @ np.abs(h2r) + np.abs(d3r).T @ dh2 + dd3r.T @ dh2
                 + gamma(N) * (np.abs(d3r).T @ np.abs(h2r)))
    out["b3"] = dd3.sum(0) + gamma(N) * np.abs(d3).sum(0)

    def back(dr, ddr, W, a, da, h):
        """delta of the layer below: (dr W) masked by h > 0, and its bound."""
        e = np.abs(dr) @ np.abs(W)
        dd = ddr @ np.abs(W) + gamma(W.shape[0]) * e
        d = (dr @ W) * (h > 0)
        if flips:
            dd = np.where(np.abs(a) <= da, e + dd, dd * (h > 0))
        else:
            dd = dd * (h > 0)
        return d, dd

    d2, dd2 = back(d3r, dd3r, W3, f["a2"], f["da2"], f["h2"])
    d2r = bf16(d2)
    dd2r = _round_gap(d2, dd2, flips)
    out["W2"] = (dd2r.T @ np.abs(h1r) + np.abs(d2r).T @ dh1 + dd2r.T @ dh1
                 + gamma(N) * (np.abs(d2r).T @ np.abs(h1r)))
    out["b2"] = dd2.sum(0) + gamma(N) * np.abs(d2).sum(0)
    d1, dd1 = back(d2r, dd2r, W2, f["a1"], f["da1"], f["h1"])
    d1r = bf16(d1)
    dd1r = _round_gap(d1, dd1, flips)
    x = f["x"]
    out["W1"] = dd1r.T @ np.abs(x) + gamma(N) * (np.abs(d1r).T @ np.abs(x))
    out["b1"] = dd1.sum(0) + gamma(N) * np.abs(d1).sum(0)
    return out


def assert_within(got, want, worst, name: str, noflip=None, axis: int | None = None, frac: float = 0.01):
    """|got - want| <= worst entry by entry (the worst case: every rounding
    decision may differ).  With `noflip`, also at most `frac` of the entries
    of every slice along `axis` (all entries when axis is None) beyond the
    bound that assumes the rounding decisions agree: a flipped decision is
    rare, and an error in one weight or bias shows up as a whole row or
    column beyond it.  Returns the largest error / worst-case bound."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    worst = np.broadcast_to(np.asarray(worst, np.float64), want.shape)
    err = np.abs(got - want)
    ratio = err / np.maximum(worst, 1e-300)
    bad = err > worst
    assert not bad.any(), (f"{name}: {int(bad.sum())} of {err.size} entries outside the worst-case bound; "
                           f"worst {float(ratio.max()):.3g} x bound at "
                           f"{np.unravel_index(int(np.argmax(ratio)), err.shape)}")
    if noflip is not None:
        nf = np.broadcast_to(np.asarray(noflip, np.float64), want.shape)
        beyond = err > nf
        fr = beyond.mean() if axis is None else beyond.mean(axis=tuple(a for a in range(err.ndim) if a != axis))
        assert np.all(fr <= frac), (f"{name}: fraction of entries beyond the no-flip bound "
                                    f"{np.max(fr):.3%} (limit {frac:.1%})")
    return float(ratio.max())
