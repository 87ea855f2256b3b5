"""CPU oracle of the learned warm start (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import this module.  It shares no code with the GPU
library.  Everything is plain numpy in float64; the bfloat16 roundings of
the GPU path are modelled by `bf16`, so the float64 products here differ
from the GPU's float32 accumulations only in summation order and width.

What is computed (the paper's Lagrangian dual, made warm-startable):

* Orbits.  The z variables of RLT2 come in orbits of six that the
  symmetry constraints (Eq. rlt2:con3) tie together: the orderings of one
  unordered set {A=(i,p), B=(j,q), C=(k,r)} of (facility, location) pairs,
  i<j<k, with p, q, r distinct.  Orbit ids run over the facility triples
  in lexicographic order, then over the ordered location triple (p, q', r'')
  with q' and r'' compressed past the smaller locations.  Members come in
  the canonical order (A,B,C),(A,C,B),(B,A,C),(B,C,A),(C,A,B),(C,B,A); member
  (P1,P2,P3) is the z variable (P1.fac, P2.fac, P3.fac, P1.loc, P2.loc,
  P3.loc).
* Multipliers.  Any v that sums to zero over every orbit (and u that sums
  to zero over every y pair) is a valid choice of Lagrange multipliers for
  those constraints (the dual of Section 3.1), so the relaxation with z
  costs -v gives a valid bound whatever v is (weak duality).  The warm start
  predicts v per orbit, projects each orbit's six values to zero sum, and
  restarts the ascent from those costs (Algorithm 1 step 1 with given
  multipliers).
* Features, a three-layer perceptron, its loss, gradients and Adam: plain
  definitions, written out below.
"""
from __future__ import annotations

import itertools

import numpy as np

FEATURES = 32          # input width (28 used, 4 zero)
USED_FEATURES = 28
OUTPUTS = 6
MEMBER_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


# ------------------------------------------------------------------ orbits --
def triples(n: int) -> np.ndarray:
    return np.array(list(itertools.combinations(range(n), 3)), dtype=np.int64).reshape(-1, 3)


def orbit_count(n: int) -> int:
    return len(triples(n)) * n * (n - 1) * (n - 2)


def decode_orbits(n: int, ids) -> np.ndarray:
    """Orbit ids -> rows (i, j, k, p, q, r), i<j<k, p, q, r distinct."""
    ids = np.asarray(ids, dtype=np.int64)
    L3 = n * (n - 1) * (n - 2)
    tri = triples(n)[ids // L3]
    rest = ids % L3
    p = rest // ((n - 1) * (n - 2))
    qq = (rest // (n - 2)) % (n - 1)
    rr = rest % (n - 2)
    q = qq + (qq >= p)
    lo, hi = np.minimum(p, q), np.maximum(p, q)
    r = rr + (rr >= lo)
    r = r + (r >= hi)
    return np.stack([tri[:, 0], tri[:, 1], tri[:, 2], p, q, r], 1)


def members(n: int, ids) -> np.ndarray:
    """(count, 6, 6): the six z variables (i,j,k,p,q,r) of each orbit."""
    o = decode_orbits(n, ids)
    fac = o[:, :3]
    loc = o[:, 3:]
    out = np.empty((len(o), 6, 6), dtype=np.int64)
    for e, (a, b, c) in enumerate(MEMBER_PERMS):
        out[:, e] = np.stack([fac[:, a], fac[:, b], fac[:, c], loc[:, a], loc[:, b], loc[:, c]], 1)
    return out


# ---------------------------------------------------------------- features --
def scales(F, D):
    """sF, sD and the multiplier scale s / (n - 2), s = sF * sD."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    n = F.shape[0]
    sF = max(1.0, float(np.abs(F).max()))
    sD = max(1.0, float(np.abs(D).max()))
    return sF, sD, sF * sD / (n - 2)


def features(F, D, B, ids) -> np.ndarray:
    """Per-orbit inputs of the perceptron (float64, 32 columns).

    With Fn = F / sF, Dn = D / sD (sF, sD the largest magnitudes, at least
    1), sym(M)_ab = (M_ab + M_ba) / 2, fa_a = sum_l (Fn_al + Fn_la) / 2n,
    dl_p likewise for Dn, Xn = (B + f_ii d_pp) / (sF sD), fbar and dbar the
    means of the off-diagonal Fn and Dn entries:
      0-5   Fn_ij Dn_pq, Fn_ji Dn_qp, Fn_ik Dn_pr, Fn_ki Dn_rp, Fn_jk Dn_qr,
            Fn_kj Dn_rq             (the RLT1 pair costs of the orbit)
      6-8   sym(Fn) of (i,j), (i,k), (j,k)
      9-11  sym(Dn) of (p,q), (p,r), (q,r)
      12-14 fa_i, fa_j, fa_k
      15-17 dl_p, dl_q, dl_r
      18-20 Xn_ip, Xn_jq, Xn_kr
      21    1 / (n - 2)
      22-24 sym(Fn) of (i,j), (i,k), (j,k) times dbar
      25-27 sym(Dn) of (p,q), (p,r), (q,r) times fbar
      28-31 zero
    """
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    B = np.zeros_like(F) if B is None else np.asarray(B, dtype=np.float64)
    n = F.shape[0]
    sF, sD, _ = scales(F, D)
    Fn = F / sF
    Dn = D / sD
    off = ~np.eye(n, dtype=bool)
    fbar = Fn[off].mean()
    dbar = Dn[off].mean()
    fa = (Fn.sum(1) + Fn.sum(0)) / (2 * n)
    dl = (Dn.sum(1) + Dn.sum(0)) / (2 * n)
    Xn = (B + np.outer(np.diag(F), np.diag(D))) / (sF * sD)
    o = decode_orbits(n, ids)
    i, j, k, p, q, r = o.T
    sf = lambda a, b: (Fn[a, b] + Fn[b, a]) / 2
    sd = lambda a, b: (Dn[a, b] + Dn[b, a]) / 2
    cols = [Fn[i, j] * Dn[p, q], Fn[j, i] * Dn[q, p], Fn[i, k] * Dn[p, r], Fn[k, i] * Dn[r, p],
            Fn[j, k] * Dn[q, r], Fn[k, j] * Dn[r, q],
            sf(i, j), sf(i, k), sf(j, k), sd(p, q), sd(p, r), sd(q, r),
            fa[i], fa[j], fa[k], dl[p], dl[q], dl[r],
            Xn[i, p], Xn[j, q], Xn[k, r], np.full(len(o), 1.0 / (n - 2)),
            sf(i, j) * dbar, sf(i, k) * dbar, sf(j, k) * dbar,
            sd(p, q) * fbar, sd(p, r) * fbar, sd(q, r) * fbar]
    X = np.zeros((len(o), FEATURES))
    X[:, :USED_FEATURES] = np.stack(cols, 1)
    return X


def targets(V, ids, scale: float) -> np.ndarray:
    """Tracked multipliers of each orbit's six members / scale, rounded to
    float32 (as the training inputs are)."""
    V = np.asarray(V)
    n = V.shape[0]
    mem = members(n, ids)
    v = V[tuple(mem.reshape(-1, 6).T)].reshape(-1, 6)
    return (v / scale).astype(np.float32)


# ---------------------------------------------------------- number formats --
def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    """Round to bfloat16, nearest with ties to even, through float32 (the
    GPU rounds its float32 values).  Returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# -------------------------------------------------------------- perceptron --
class Params:
    """W1 (256 x 32), b1, W2 (256 x 256), b2, W3 (6 x 256), b3; float32
    values held as float64."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, W1, b1, W2, b2, W3, b3):
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = (f32(a) for a in (W1, b1, W2, b2, W3, b3))

    def tensors(self):
        return [getattr(self, k) for k in self.NAMES]


def forward(P: Params, X, rounding: bool = True):
    """y = W3 h2 + b3, h2 = relu(W2 h1 + b2), h1 = relu(W1 x + b1), with
    every matrix-product operand rounded to bfloat16 when `rounding`
    (inputs, weights, hidden activations) and float64 accumulation."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(X)
    h1 = np.maximum(x @ r(P.W1).T + P.b1, 0.0)
    h1r = r(h1)
    h2 = np.maximum(h1r @ r(P.W2).T + P.b2, 0.0)
    h2r = r(h2)
    y = h2r @ r(P.W3).T + P.b3
    return y, {"x": x, "h1": h1, "h1r": h1r, "h2": h2, "h2r": h2r}


def project(y) -> np.ndarray:
    """Zero-sum projection of each row of six values."""
    y = np.asarray(y, dtype=np.float64)
    return y - y.mean(axis=1, keepdims=True)


def loss(y, t) -> float:
    """Mean squared error of the projected outputs against the targets."""
    d = project(y) - np.asarray(t, dtype=np.float64)
    return float((d * d).mean())


def gradients(P: Params, X, T, rounding: bool = True):
    """Gradients of `loss(forward(P, X)[0], T)` with respect to W1..b3.

    With rounding, the backward pass rounds its product operands too: the
    output error delta3 = projection of 2 (proj(y) - t) / (6 N), delta2 =
    (delta3 W3) masked by h2 > 0, delta1 = (delta2 W2) masked by h1 > 0, each
    rounded to bfloat16 before it enters a product; bias gradients sum the
    unrounded deltas.  Without rounding this is the exact gradient."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(P, X, rounding)
    N = y.shape[0]
    g = 2.0 * (project(y) - np.asarray(T, dtype=np.float64)) / (6.0 * N)
    d3 = project(g)
    d3r = r(d3)
    gW3 = d3r.T @ c["h2r"]
    gb3 = d3.sum(0)
    d2 = (d3r @ r(P.W3)) * (c["h2"] > 0)
    d2r = r(d2)
    gW2 = d2r.T @ c["h1r"]
    gb2 = d2.sum(0)
    d1 = (d2r @ r(P.W2)) * (c["h1"] > 0)
    d1r = r(d1)
    gW1 = d1r.T @ c["x"]
    gb1 = d1.sum(0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def adam_step(w, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) at step t >= 1; returns
    the new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# -------------------------------------------------------------- warm start --
def multipliers_from_outputs(n: int, y, scale: float) -> np.ndarray:
    """Dense n^6 multipliers v from per-orbit outputs y (all orbits, id
    order): v_e = (y_e - mean) * scale, the mean a left-to-right sum of the
    six float32 outputs divided by 6, in float64."""
    y = np.asarray(y, dtype=np.float32).astype(np.float64)
    ids = np.arange(orbit_count(n))
    mean = (((((y[:, 0] + y[:, 1]) + y[:, 2]) + y[:, 3]) + y[:, 4]) + y[:, 5]) / 6.0
    v = (y - mean[:, None]) * scale
    V = np.zeros((n,) * 6)
    mem = members(n, ids)
    V[tuple(mem.reshape(-1, 6).T)] = v.reshape(-1)
    return V
