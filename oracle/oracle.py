"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import this module.  It shares no code with the GPU
library; the two meet only in the seeded instance generator.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build_oracle

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(build_oracle.SRC):
            build_oracle.build(force=True)
        L = C.CDLL(path)
        L.orc_lap.argtypes = [C.c_int, _dp, _dp, _dp, _ip, _dp, C.POINTER(C.c_longlong)]
        L.orc_qap_cost.argtypes = [C.c_int, _dp, _dp, _dp, _ip]
        L.orc_qap_cost.restype = C.c_double
        L.orc_bruteforce.argtypes = [C.c_int, _dp, _dp, _dp, _ip, _dp]
        L.orc_glb.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_da_create.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_da_create.restype = C.c_void_p
        L.orc_da_from_arrays.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.orc_da_from_arrays.restype = C.c_void_p
        L.orc_da_free.argtypes = [C.c_void_p]
        for name in ("orc_da_sweep", "orc_da_zphase", "orc_da_yequal", "orc_da_yphase",
                     "orc_da_xphase", "orc_da_iterate"):
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_da_run.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_da_proven.argtypes = [C.c_void_p]
        L.orc_da_n.argtypes = [C.c_void_p]
        L.orc_da_t.argtypes = [C.c_void_p]
        L.orc_da_lb.argtypes = [C.c_void_p]
        L.orc_da_lb.restype = C.c_double
        L.orc_da_ub.argtypes = [C.c_void_p]
        L.orc_da_ub.restype = C.c_double
        L.orc_da_steps.argtypes = [C.c_void_p]
        L.orc_da_steps.restype = C.c_longlong
        L.orc_da_trace.argtypes = [C.c_void_p, _dp, C.c_int]
        L.orc_da_perms.argtypes = [C.c_void_p, _ip, _ip]
        L.orc_da_export.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_da_z_tiles.argtypes = [C.c_void_p, C.c_int, _ip, _dp]
        L.orc_da_identity.argtypes = [C.c_void_p, _ip]
        L.orc_da_identity.restype = C.c_double
        L.orc_da_min_entries.argtypes = [C.c_void_p, _dp]
        L.orc_rule3_order.argtypes = [C.c_int, _dp, _ip]
        L.orc_da_fold.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_da_fold.restype = C.c_void_p
        L.orc_da_offset.argtypes = [C.c_void_p]
        L.orc_da_offset.restype = C.c_double
        L.orc_bnb.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, C.c_int, C.c_double,
                              C.c_double, _ip, _dp, C.POINTER(C.c_longlong)]
        L.orc_glb_bnb.argtypes = [C.c_int, _dp, _dp, _dp, C.c_double, _ip, _dp,
                                  C.POINTER(C.c_longlong)]
        L.orc_da_create_xy.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_da_create_xy.restype = C.c_void_p
        L.orc_da_iter0_xy.argtypes = [C.c_void_p]
        L.orc_iter1_tile.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_da_track.argtypes = [C.c_void_p]
        L.orc_da_set_half.argtypes = [C.c_void_p]
        L.orc_da_set_two_phase.argtypes = [C.c_void_p]
        L.orc_da_pool.argtypes = [C.c_void_p]
        L.orc_da_set_slow.argtypes = [C.c_void_p]
        L.orc_splitmix64.argtypes = [C.c_ulonglong, C.c_ulonglong]
        L.orc_splitmix64.restype = C.c_ulonglong
        L.orc_sa_uniform.argtypes = [C.c_ulonglong, C.c_ulonglong]
        L.orc_sa_uniform.restype = C.c_double
        L.orc_sa_exp.argtypes = [C.c_double]
        L.orc_sa_exp.restype = C.c_double
        L.orc_da_set_annealing.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int,
                                           C.c_ulonglong]
        L.orc_da_type4.argtypes = [C.c_void_p, C.c_int]
        L.orc_da_sa_accepted.argtypes = [C.c_void_p]
        L.orc_da_sa_accepted.restype = C.c_longlong
        L.orc_da_multipliers.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_da_from_multipliers.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_da_from_multipliers.restype = C.c_void_p
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def max_threads() -> int:
    return int(lib().orc_max_threads())


FULL = (5.0 / 6.0, 1.0, 1.0, 1.0 / 5.0, 0.5)
# HALF scheme of Section 5: upper-member kz = 2/3, ky = kx = 1, upper share
# phi = 1/2, y-pair 1/2; the trailing 1 selects the scheme (orc_da_set_half)
HALF = (2.0 / 3.0, 1.0, 1.0, 0.5, 0.5, 1.0)


def lap(M):
    """Hungarian LAP.  Returns (theta, u, v, row_of_col, pi, steps)."""
    M = _f64(M)
    m = M.shape[0]
    u = np.zeros(m)
    v = np.zeros(m)
    rc = np.zeros(m, dtype=np.int32)
    th = C.c_double(0.0)
    st = C.c_longlong(0)
    rc_ = lib().orc_lap(m, _d(M), _d(u), _d(v), _i(rc), C.byref(th), C.byref(st))
    if rc_ != 0:
        raise ValueError("bad LAP size")
    pi = (M - u[:, None]) - v[None, :]
    return th.value, u, v, rc, pi, st.value


def qap_cost(F, D, B, perm) -> float:
    F, D, B = _f64(F), _f64(D), _f64(B)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    return float(lib().orc_qap_cost(F.shape[0], _d(F), _d(D), _d(B), _i(perm)))


def bruteforce(F, D, B):
    F, D, B = _f64(F), _f64(D), _f64(B)
    n = F.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    c = C.c_double(0.0)
    if lib().orc_bruteforce(n, _d(F), _d(D), _d(B), _i(perm), C.byref(c)) != 0:
        raise ValueError("n too large for brute force")
    return c.value, perm


def glb(F, D, B) -> float:
    F, D, B = _f64(F), _f64(D), _f64(B)
    g = C.c_double(0.0)
    lib().orc_glb(F.shape[0], _d(F), _d(D), _d(B), C.byref(g))
    return g.value


def rule3_order(F):
    F = _f64(F)
    o = np.zeros(F.shape[0], dtype=np.int32)
    lib().orc_rule3_order(F.shape[0], _d(F), _i(o))
    return o


class DualAscent:
    """The F1 RLT2 dual ascent on dense reduced-cost arrays."""

    def __init__(self, F, D, B=None, params=FULL, _handle=None, two_phase=False, slow=False):
        F, D = _f64(F), _f64(D)
        self.n = F.shape[0]
        B = np.zeros_like(F) if B is None else _f64(B)
        self._keep = (F, D, B)
        P = _f64(params)
        self._params = P
        h = _handle if _handle is not None else lib().orc_da_create(self.n, _d(F), _d(D), _d(B), _d(P[:5]))
        if not h:
            raise ValueError("oracle: bad instance")
        self.h = C.c_void_p(h)
        self.half = len(P) > 5 and P[5] == 1.0
        if self.half and lib().orc_da_set_half(self.h) != 0:
            raise ValueError("oracle: HALF needs zero lower z costs and no tracking")
        self.two_phase = bool(two_phase)
        if self.two_phase and lib().orc_da_set_two_phase(self.h) != 0:
            raise ValueError("oracle: F2 is not combined with HALF or tracking")
        self.slow = bool(slow)
        if self.slow and lib().orc_da_set_slow(self.h) != 0:
            raise ValueError("oracle: S1 needs a fresh FULL state without annealing")

    @classmethod
    def from_arrays(cls, F, D, B, params, LB, X, Y, Z):
        F, D, B = _f64(F), _f64(D), _f64(B)
        X, Y, Z = _f64(X), _f64(Y), _f64(Z)
        P = _f64(params)
        h = lib().orc_da_from_arrays(F.shape[0], _d(F), _d(D), _d(B), _d(P), float(LB),
                                     _d(X), _d(Y), _d(Z))
        return cls(F, D, B, params, _handle=h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().orc_da_free(h)
            self.h = None

    # phases
    def sweep(self):
        lib().orc_da_sweep(self.h)

    def zphase(self):
        lib().orc_da_zphase(self.h)

    def pool(self):
        """F2's pooling of the orbit slacks (S_N onto S_B)."""
        lib().orc_da_pool(self.h)

    def set_annealing(self, t0: float, kappa_max: float = 0.25, cool: float = 0.99, period: int = 100,
                      seed: int = 0):
        """Type 4 ascent with simulated annealing after every iteration t >= 1
        (t0 <= 0 turns it off)."""
        if lib().orc_da_set_annealing(self.h, float(t0), float(kappa_max), float(cool), int(period),
                                      int(seed)) != 0:
            raise ValueError("oracle: bad annealing parameters, or tracking is on")

    def type4(self, it: int) -> bool:
        """One Type 4 step for iteration index `it` on the current state."""
        return bool(lib().orc_da_type4(self.h, int(it)))

    @property
    def sa_accepted(self) -> int:
        return int(lib().orc_da_sa_accepted(self.h))

    def yequal(self):
        lib().orc_da_yequal(self.h)

    def yphase(self):
        lib().orc_da_yphase(self.h)

    def xphase(self):
        lib().orc_da_xphase(self.h)

    def iterate(self):
        lib().orc_da_iterate(self.h)

    def run(self, iters: int, min_gap: float = 0.0) -> int:
        return int(lib().orc_da_run(self.h, int(iters), float(min_gap)))

    @property
    def t(self) -> int:
        return int(lib().orc_da_t(self.h))

    @property
    def LB(self) -> float:
        return float(lib().orc_da_lb(self.h))

    @property
    def UB(self) -> float:
        return float(lib().orc_da_ub(self.h))

    @property
    def steps(self) -> int:
        return int(lib().orc_da_steps(self.h))

    def proven(self) -> bool:
        return bool(lib().orc_da_proven(self.h))

    def trace(self):
        cap = max(1, self.t)
        out = np.zeros(cap)
        k = lib().orc_da_trace(self.h, _d(out), cap)
        return out[:k]

    def perms(self):
        a = np.zeros(self.n, dtype=np.int32)
        b = np.zeros(self.n, dtype=np.int32)
        lib().orc_da_perms(self.h, _i(a), _i(b))
        return a, b

    def export(self, with_z: bool = True):
        """Dense X (n^2), Y (n^4) and Z (n^6, None without with_z)."""
        n = self.n
        X = np.zeros((n, n))
        Y = np.zeros((n,) * 4)
        Z = np.zeros((n,) * 6) if with_z else None
        lib().orc_da_export(self.h, _d(X), _d(Y), None if Z is None else _d(Z))
        return X, Y, Z

    def z_tiles(self, picks):
        """The z reduced costs of tiles (i, j, p, q): array (len, m, m), rows
        k and columns r over the remaining indices in ascending order."""
        m = self.n - 2
        ijpq = np.ascontiguousarray(np.asarray(picks, dtype=np.int32).reshape(-1, 4))
        out = np.zeros((len(ijpq), m, m))
        if lib().orc_da_z_tiles(self.h, len(ijpq), _i(ijpq), _d(out)) != 0:
            raise ValueError("z_tiles: bad tile")
        return out

    def identity(self, perm) -> float:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        return float(lib().orc_da_identity(self.h, _i(perm)))

    def fold(self, l: int, s: int):
        """Child state after fixing local facility l to local location s (a
        self-contained QAP on the free indices plus a constant offset)."""
        F, D, B = self._keep
        keep_f = [a for a in range(self.n) if a != l]
        keep_l = [a for a in range(self.n) if a != s]
        Fc = _f64(F[np.ix_(keep_f, keep_f)])
        Dc = _f64(D[np.ix_(keep_l, keep_l)])
        Bc = _f64((B[np.ix_(keep_f, keep_l)] + np.outer(F[keep_f, l], D[keep_l, s]))
                  + np.outer(F[l, keep_f], D[s, keep_l]))
        h = lib().orc_da_fold(self.h, int(l), int(s))
        if not h:
            raise ValueError("fold: bad arguments")
        return DualAscent(Fc, Dc, Bc, tuple(self._params), _handle=h)

    def track(self):
        if lib().orc_da_track(self.h) != 0:
            raise MemoryError("tracking arrays")

    def multipliers(self):
        n = self.n
        V = np.zeros((n,) * 6)
        U = np.zeros((n,) * 4)
        lib().orc_da_multipliers(self.h, _d(V), _d(U))
        return V, U

    @classmethod
    def from_multipliers(cls, F, D, B, params, V, U):
        F, D = _f64(F), _f64(D)
        B = np.zeros_like(F) if B is None else _f64(B)
        P = _f64(params)
        Vp = None if V is None else _d(_f64(V))
        Up = None if U is None else _d(_f64(U))
        keepV = None if V is None else _f64(V)
        keepU = None if U is None else _f64(U)
        h = lib().orc_da_from_multipliers(F.shape[0], _d(F), _d(D), _d(B), _d(P),
                                          None if keepV is None else _d(keepV),
                                          None if keepU is None else _d(keepU))
        return cls(F, D, B, params, _handle=h)

    @property
    def offset(self) -> float:
        return float(lib().orc_da_offset(self.h))

    def min_entries(self):
        out = np.zeros(3)
        lib().orc_da_min_entries(self.h, _d(out))
        return out


def bnb(F, D, B=None, params=FULL, node_iters=100, window=25, min_improve=2e-4,
        ub0=float("inf")):
    F, D = _f64(F), _f64(D)
    n = F.shape[0]
    B = np.zeros_like(F) if B is None else _f64(B)
    P = _f64(params)
    perm = np.zeros(n, dtype=np.int32)
    obj = C.c_double(0.0)
    st = (C.c_longlong * 3)()
    rc = lib().orc_bnb(n, _d(F), _d(D), _d(B), _d(P), int(node_iters), int(window),
                       float(min_improve), float(ub0), _i(perm), C.byref(obj), st)
    if rc != 0:
        raise ValueError("oracle B&B: bad size")
    return obj.value, perm, {"nodes": st[0], "da_iters": st[1], "enumerated": st[2]}


def glb_bnb(F, D, B=None, ub0=float("inf")):
    F, D = _f64(F), _f64(D)
    n = F.shape[0]
    B = np.zeros_like(F) if B is None else _f64(B)
    perm = np.zeros(n, dtype=np.int32)
    obj = C.c_double(0.0)
    nodes = C.c_longlong(0)
    rc = lib().orc_glb_bnb(n, _d(F), _d(D), _d(B), float(ub0), _i(perm), C.byref(obj),
                           C.byref(nodes))
    if rc != 0:
        raise ValueError("GLB B&B: bad size")
    return obj.value, perm, nodes.value


class Iter0XY:
    """Iteration 0 without the (identically zero) z level, and single tiles of
    the iteration-1 Z-LAPs; for sizes whose n^6 array does not fit a test."""

    def __init__(self, F, D, B=None, params=FULL):
        F, D = _f64(F), _f64(D)
        self.n = F.shape[0]
        B = np.zeros_like(F) if B is None else _f64(B)
        self._keep = (F, D, B)
        P = _f64(params)
        h = lib().orc_da_create_xy(self.n, _d(F), _d(D), _d(B), _d(P[:5]))
        if not h:
            raise ValueError("oracle: bad instance")
        self.h = C.c_void_p(h)
        self.half = len(P) > 5 and P[5] == 1.0
        if self.half and lib().orc_da_set_half(self.h) != 0:
            raise ValueError("oracle: HALF switch refused")
        if lib().orc_da_iter0_xy(self.h) != 0:
            raise RuntimeError("iteration 0 failed")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().orc_da_free(h)
            self.h = None

    @property
    def LB(self) -> float:
        return float(lib().orc_da_lb(self.h))

    @property
    def UB(self) -> float:
        return float(lib().orc_da_ub(self.h))

    def xy(self):
        n = self.n
        X = np.zeros((n, n))
        Y = np.zeros((n,) * 4)
        lib().orc_da_export(self.h, _d(X), _d(Y), None)
        return X, Y

    def tile1(self, i, j, p, q):
        m = self.n - 2
        M = np.zeros((m, m))
        pi = np.zeros((m, m))
        th = C.c_double(0.0)
        if lib().orc_iter1_tile(self.h, i, j, p, q, _d(M), _d(pi), C.byref(th)) != 0:
            raise ValueError("bad tile")
        return M, pi, th.value


def splitmix64(seed: int, c: int) -> int:
    return int(lib().orc_splitmix64(int(seed), int(c)))


def sa_uniform(seed: int, c: int) -> float:
    return float(lib().orc_sa_uniform(int(seed), int(c)))


def sa_exp(x: float) -> float:
    return float(lib().orc_sa_exp(float(x)))
