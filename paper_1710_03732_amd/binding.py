"""ctypes binding of the C ABI in include/qap_rlt2.h (argument marshalling
only; every step of the dual ascent runs in the HIP library).

The shared library is built in-tree by ``paper_1710_03732_amd/build.py``;
importing a handle without it raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqaprlt2.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qap_rlt2.h")

QAP_OK = 0
ERRORS = {-1: "QAP_EINVAL", -2: "QAP_ENOMEM", -3: "QAP_EDEVICE", -4: "QAP_ESTATE",
          -5: "QAP_EUNSUPPORTED"}

_alloc_fn = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_free_fn = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class QapParams(C.Structure):
    _fields_ = [("kappa_z", C.c_double), ("kappa_y", C.c_double), ("kappa_x", C.c_double),
                ("phi_z", C.c_double), ("phi_y", C.c_double), ("min_gap", C.c_double),
                ("device", C.c_int), ("zlap_lanes", C.c_int), ("zlap_cols", C.c_int),
                ("timing", C.c_int), ("scheme", C.c_int), ("two_phase", C.c_int), ("slow", C.c_int),
                ("alloc", _alloc_fn),
                ("free_fn", _free_fn), ("alloc_ctx", C.c_void_p)]


SCHEME_FULL = 0
SCHEME_HALF = 1


class QapDaStats(C.Structure):
    _fields_ = [("iterations_done", C.c_int), ("t", C.c_int), ("lb", C.c_double),
                ("ub", C.c_double), ("gap", C.c_double), ("proven", C.c_int), ("sa_steps", C.c_int),
                ("laps", C.c_longlong), ("dijkstra_steps", C.c_longlong), ("seconds", C.c_double),
                ("ms_sweep", C.c_double), ("ms_zlap", C.c_double), ("ms_ylap", C.c_double),
                ("ms_xlap", C.c_double), ("best_lb", C.c_double)]


class QapSaParams(C.Structure):
    _fields_ = [("t0", C.c_double), ("kappa_max", C.c_double), ("cool", C.c_double),
                ("period", C.c_int), ("pad", C.c_int), ("seed", C.c_uint64)]


class QapBnbParams(C.Structure):
    _fields_ = [("batch", C.c_int), ("node_iters", C.c_int), ("window", C.c_int),
                ("root_iters", C.c_int), ("min_improve", C.c_double), ("ub0", C.c_double),
                ("enum_below", C.c_int), ("rule", C.c_int), ("depth_cap", C.c_int), ("symmetry", C.c_int)]


class QapBnbStats(C.Structure):
    _fields_ = [("nodes", C.c_longlong), ("da_iters", C.c_longlong), ("batches", C.c_longlong),
                ("enumerated", C.c_longlong), ("seconds", C.c_double), ("symmetric_skipped", C.c_longlong),
                ("automorphisms", C.c_longlong), ("node_bytes", C.c_double)]


class QapBatchParams(C.Structure):
    _fields_ = [("iters", C.c_int), ("window", C.c_int), ("min_improve", C.c_double),
                ("ub_cut", C.c_double), ("zlap_lanes", C.c_int), ("reserved", C.c_int)]


class QapBatchStats(C.Structure):
    _fields_ = [("iterations", C.c_longlong), ("stopped", C.c_int), ("fathomed", C.c_int),
                ("window_stops", C.c_int), ("compactions", C.c_int), ("seconds", C.c_double)]


class QapStateHeader(C.Structure):
    _fields_ = [("n", C.c_int), ("t", C.c_int), ("lb", C.c_double), ("ub", C.c_double),
                ("checksum", C.c_uint64)]


class QapAdamParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class QapWarmStats(C.Structure):
    _fields_ = [("orbits", C.c_longlong), ("scale", C.c_double), ("gain", C.c_double), ("ms_mlp", C.c_double),
                ("ms_write", C.c_double), ("seconds", C.c_double), ("mlp_flops", C.c_double)]


MLP_PARAMS = 75782   # W1 [256][32], b1, W2 [256][256], b2, W3 [6][256], b3
MLP_SHAPES = (("W1", (256, 32)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (6, 256)), ("b3", (6,)))


_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_lib = None

EXPORTED = ("qap_version", "qap_default_params", "qap_workspace_bytes", "qap_rlt2_init",
            "qap_destroy", "qap_dual_ascent", "qap_get_trace", "qap_get_assignment",
            "qap_export_state", "qap_export_z_tiles", "qap_import_state", "qap_set_stream", "qap_bnb_solve",
            "qap_lap_batch", "qap_last_error", "qap_fold_child", "qap_batch_dual_ascent",
            "qap_batch_dual_ascent_static",
            "qap_node_status", "qap_track", "qap_get_multipliers", "qap_set_multipliers",
            "qap_orbit_count", "qap_multiplier_scale", "qap_orbit_features", "qap_orbit_targets",
            "qap_warm_start_outputs", "qap_mlp_create", "qap_mlp_destroy", "qap_mlp_set_stream",
            "qap_mlp_get_params", "qap_mlp_forward", "qap_mlp_gradients", "qap_mlp_train_step",
            "qap_orbit_outputs", "qap_warm_start", "qap_set_allocator", "qap_zlap_mapping",
            "qap_set_annealing", "qap_location_automorphisms")


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; run paper_1710_03732_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.qap_version.restype = C.c_char_p
        L.qap_default_params.argtypes = [C.POINTER(QapParams)]
        L.qap_workspace_bytes.argtypes = [C.c_int, C.POINTER(QapParams)]
        L.qap_workspace_bytes.restype = C.c_size_t
        L.qap_rlt2_init.argtypes = [_dp, _dp, _dp, C.c_int, C.POINTER(QapParams), C.POINTER(C.c_void_p)]
        L.qap_destroy.argtypes = [C.c_void_p]
        L.qap_set_annealing.argtypes = [C.c_void_p, C.c_void_p]
        L.qap_location_automorphisms.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_void_p, C.POINTER(C.c_int)]
        L.qap_zlap_mapping.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)]
        L.qap_dual_ascent.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, C.POINTER(QapDaStats)]
        L.qap_get_trace.argtypes = [C.c_void_p, _dp, C.c_int, C.POINTER(C.c_int)]
        L.qap_get_assignment.argtypes = [C.c_void_p, _i32p, _i32p]
        L.qap_export_state.argtypes = [C.c_void_p, C.POINTER(QapStateHeader), _dp, _dp, _dp]
        L.qap_export_z_tiles.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int, _dp]
        L.qap_import_state.argtypes = [C.c_void_p, C.POINTER(QapStateHeader), _dp, _dp, _dp]
        L.qap_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.qap_bnb_solve.argtypes = [C.c_void_p, C.POINTER(QapBnbParams), _i32p, _dp,
                                    C.POINTER(QapBnbStats)]
        L.qap_lap_batch.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.qap_fold_child.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
        L.qap_batch_dual_ascent.argtypes = [C.POINTER(C.c_void_p), C.c_int,
                                            C.POINTER(QapBatchParams), C.POINTER(QapBatchStats)]
        L.qap_batch_dual_ascent_static.argtypes = [C.POINTER(C.c_void_p), C.c_int,
                                                   C.POINTER(QapBatchParams), C.POINTER(QapBatchStats)]
        L.qap_node_status.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
        L.qap_last_error.argtypes = [C.c_void_p]
        L.qap_last_error.restype = C.c_char_p
        vp = C.c_void_p
        L.qap_track.argtypes = [vp, C.c_int]
        L.qap_get_multipliers.argtypes = [vp, _dp, _dp]
        L.qap_set_multipliers.argtypes = [vp, _dp, _dp]
        L.qap_orbit_count.argtypes = [C.c_int, C.POINTER(C.c_int64)]
        L.qap_multiplier_scale.argtypes = [vp, _dp]
        L.qap_orbit_features.argtypes = [vp, vp, C.c_int64, vp]
        L.qap_orbit_targets.argtypes = [vp, vp, C.c_int64, C.c_double, vp]
        L.qap_warm_start_outputs.argtypes = [vp, vp, C.c_double]
        L.qap_mlp_create.argtypes = [C.POINTER(C.c_float), C.c_int, vp, C.POINTER(vp)]
        L.qap_mlp_destroy.argtypes = [vp]
        L.qap_mlp_set_stream.argtypes = [vp, vp]
        L.qap_mlp_get_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.qap_mlp_forward.argtypes = [vp, vp, C.c_int, vp]
        L.qap_mlp_gradients.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_float), _dp]
        L.qap_mlp_train_step.argtypes = [vp, vp, vp, C.c_int, C.POINTER(QapAdamParams), _dp]
        L.qap_orbit_outputs.argtypes = [vp, vp, vp]
        L.qap_warm_start.argtypes = [vp, vp, C.c_double, C.POINTER(QapWarmStats)]
        L.qap_set_allocator.argtypes = [vp, _alloc_fn, _free_fn, vp]
        _lib = L
    return _lib


class QapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(code, h=None):
    if code != QAP_OK:
        msg = lib().qap_last_error(h).decode(errors="replace")
        raise QapError(code, msg)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a):
    return a.ctypes.data_as(_dp)


def default_params(**kw) -> QapParams:
    p = QapParams()
    _check(lib().qap_default_params(C.byref(p)))
    names = {f[0] for f in QapParams._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown qap_params field {k!r}")
        setattr(p, k, v)
    return p


def half_params(**kw) -> QapParams:
    """The HALF preset of Section 5: kappa_z = 2/3, kappa_y = kappa_x = 1,
    phi_z = phi_y = 1/2, scalar Z-LAP mapping."""
    base = dict(kappa_z=2.0 / 3.0, kappa_y=1.0, kappa_x=1.0, phi_z=0.5, phi_y=0.5,
                zlap_lanes=-1, scheme=SCHEME_HALF)
    base.update(kw)
    return default_params(**base)


def version() -> str:
    return lib().qap_version().decode()


def workspace_bytes(n: int) -> int:
    return int(lib().qap_workspace_bytes(int(n), None))


def tile_count(n: int) -> int:
    return n * n * (n - 1) * (n - 1)


class DualAscent:
    """Handle of one RLT2 dual-ascent state on the GPU."""

    def __init__(self, F, D, B=None, params: QapParams | None = None, _handle=None, _n=None,
                 _parent=None, **kw):
        if _handle is not None:
            self.h = _handle
            self.n = _n
            self.T = tile_count(_n)
            self.m = _n - 2
            self.params = _parent.params
            self._parent = _parent  # children share the parent's stream
            return
        F, D = _f64(F), _f64(D)
        n = F.shape[0]
        self.n = n
        Bp = None if B is None else _f64(B)
        if params is None:
            params = default_params(**kw)
        self.params = params
        h = C.c_void_p()
        code = lib().qap_rlt2_init(_dptr(F), _dptr(D), None if Bp is None else _dptr(Bp), n,
                                   C.byref(params), C.byref(h))
        _check(code)
        self.h = h
        self.T = tile_count(n)
        self.m = n - 2

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().qap_destroy(self.h)
        self.h = None

    def zlap_mapping(self):
        """(lanes, cols, tuned_us) of the Z-LAP mapping in use; lanes -1 / -2
        mean one / two LAPs per wavefront; tuned_us is -1 when the mapping
        was requested or not yet measured (see qap_zlap_mapping)."""
        lanes, cols, us = C.c_int(0), C.c_int(0), C.c_double(0.0)
        _check(lib().qap_zlap_mapping(self.h, C.byref(lanes), C.byref(cols), C.byref(us)), self.h)
        return lanes.value, cols.value, us.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, iters: int):
        lb = C.c_double(0.0)
        alpha = np.zeros(self.n)
        beta = np.zeros(self.n)
        st = QapDaStats()
        _check(lib().qap_dual_ascent(self.h, int(iters), C.byref(lb), _dptr(alpha), _dptr(beta),
                                     C.byref(st)), self.h)
        return {"lb": lb.value, "alpha": alpha, "beta": beta, "iterations_done": st.iterations_done,
                "t": st.t, "ub": st.ub, "gap": st.gap, "proven": bool(st.proven), "laps": st.laps,
                "dijkstra_steps": st.dijkstra_steps, "seconds": st.seconds,
                "ms_sweep": st.ms_sweep, "ms_zlap": st.ms_zlap, "ms_ylap": st.ms_ylap,
                "ms_xlap": st.ms_xlap, "best_lb": st.best_lb, "sa_steps": st.sa_steps}

    def set_annealing(self, t0: float, kappa_max: float = 0.25, cool: float = 0.99, period: int = 100,
                      seed: int = 0):
        """Type 4 steps with annealing after every iteration t >= 1 (Section 5's
        schedule by default); t0 <= 0 turns them off."""
        p = QapSaParams(float(t0), float(kappa_max), float(cool), int(period), 0, int(seed))
        _check(lib().qap_set_annealing(self.h, C.byref(p)), self.h)

    def trace(self):
        n = C.c_int(0)
        _check(lib().qap_get_trace(self.h, None, 0, C.byref(n)), self.h)
        out = np.zeros(max(1, n.value))
        _check(lib().qap_get_trace(self.h, _dptr(out), n.value, C.byref(n)), self.h)
        return out[:n.value]

    def assignment(self):
        a = np.zeros(self.n, dtype=np.int32)
        b = np.zeros(self.n, dtype=np.int32)
        _check(lib().qap_get_assignment(self.h, a.ctypes.data_as(_i32p), b.ctypes.data_as(_i32p)),
               self.h)
        return a, b

    def export_state(self, with_z: bool = True):
        hdr = QapStateHeader()
        x = np.zeros(self.n * self.n)
        y = np.zeros(self.T)
        z = np.zeros(self.T * self.m * self.m) if with_z else None
        _check(lib().qap_export_state(self.h, C.byref(hdr), _dptr(x), _dptr(y),
                                      None if z is None else _dptr(z)), self.h)
        return hdr, x, y, z

    def export_tiles(self, tiles):
        tiles = np.ascontiguousarray(tiles, dtype=np.int64)
        out = np.zeros((len(tiles), self.m, self.m))
        _check(lib().qap_export_z_tiles(self.h, tiles.ctypes.data_as(C.POINTER(C.c_int64)),
                                        len(tiles), _dptr(out)), self.h)
        return out

    def import_state(self, hdr, x, y, z):
        x, y, z = _f64(x), _f64(y), _f64(z)
        _check(lib().qap_import_state(self.h, C.byref(hdr), _dptr(x), _dptr(y), _dptr(z)), self.h)

    def fold(self, l: int, s: int) -> "DualAscent":
        """Child node fixing facility l to location s (0-based, this
        handle's own indices), warm-started from the current reduced costs."""
        h = C.c_void_p()
        _check(lib().qap_fold_child(self.h, int(l), int(s), C.byref(h)), self.h)
        return DualAscent(None, None, _handle=h, _n=self.n - 1, _parent=self)

    def status(self):
        t = C.c_int(0)
        lb = C.c_double(0.0)
        ub = C.c_double(0.0)
        stopped = C.c_int(0)
        reason = C.c_int(0)
        _check(lib().qap_node_status(self.h, C.byref(t), C.byref(lb), C.byref(ub),
                                     C.byref(stopped), C.byref(reason)), self.h)
        return {"t": t.value, "lb": lb.value, "ub": ub.value, "stopped": bool(stopped.value),
                "reason": reason.value}

    def set_stream(self, stream_handle: int):
        _check(lib().qap_set_stream(self.h, C.c_void_p(stream_handle)), self.h)

    def bnb_solve(self, batch=256, node_iters=100, window=25, root_iters=0, min_improve=2e-4,
                  ub0=float("inf"), enum_below=3, rule=3, depth_cap=0, symmetry=0):
        p = QapBnbParams(batch, node_iters, window, root_iters, min_improve, ub0, enum_below, rule,
                         depth_cap, symmetry)
        perm = np.zeros(self.n, dtype=np.int32)
        obj = C.c_double(0.0)
        st = QapBnbStats()
        _check(lib().qap_bnb_solve(self.h, C.byref(p), perm.ctypes.data_as(_i32p), C.byref(obj),
                                   C.byref(st)), self.h)
        return obj.value, perm, {"nodes": st.nodes, "da_iters": st.da_iters,
                                 "batches": st.batches, "enumerated": st.enumerated,
                                 "seconds": st.seconds, "symmetric_skipped": st.symmetric_skipped,
                                 "automorphisms": st.automorphisms, "node_bytes": st.node_bytes}


    # ---- multipliers and the learned warm start ---------------------------
    def track(self, on: bool = True):
        _check(lib().qap_track(self.h, 1 if on else 0), self.h)

    def multipliers(self):
        """Tracked (v, u) in the z and y layouts (host float64)."""
        v = np.zeros(self.T * self.m * self.m)
        u = np.zeros(self.T)
        _check(lib().qap_get_multipliers(self.h, _dptr(v), _dptr(u)), self.h)
        return v, u

    def set_multipliers(self, v=None, u=None):
        vv = None if v is None else _f64(v).reshape(-1)
        uu = None if u is None else _f64(u).reshape(-1)
        _check(lib().qap_set_multipliers(self.h, None if vv is None else _dptr(vv),
                                         None if uu is None else _dptr(uu)), self.h)

    def set_allocator(self, alloc=None, free=None):
        """Route later allocations (tracking arrays, learned-call buffers)
        through Python callables alloc(nbytes) -> int and free(ptr), e.g.
        torch's caching allocator; None restores hipMalloc."""
        # the library may still call the current callbacks (it refuses the
        # change while tracking arrays are live): drop them only on success
        if alloc is None:
            _check(lib().qap_set_allocator(self.h, _alloc_fn(), _free_fn(), None), self.h)
            self._alloc_cbs = None
            return
        a = _alloc_fn(lambda nbytes, ctx: alloc(nbytes))
        f = _free_fn(lambda ptr, ctx: free(ptr))
        _check(lib().qap_set_allocator(self.h, a, f, None), self.h)
        self._alloc_cbs = (a, f)  # keep the callbacks alive while the library holds them

    def multiplier_scale(self) -> float:
        s = C.c_double(0.0)
        _check(lib().qap_multiplier_scale(self.h, C.byref(s)), self.h)
        return s.value

    def orbit_features(self, ids):
        """ids: int64 CUDA tensor; returns a float32 CUDA tensor (count, 32)."""
        import torch

        ids = _device_tensor(ids, torch.int64, "ids")
        x = torch.empty((ids.numel(), 32), dtype=torch.float32, device=ids.device)
        _check(lib().qap_orbit_features(self.h, C.c_void_p(ids.data_ptr()), ids.numel(),
                                        C.c_void_p(x.data_ptr())), self.h)
        return x

    def orbit_targets(self, ids, scale: float, out=None):
        import torch

        ids = _device_tensor(ids, torch.int64, "ids")
        if out is not None:
            t = _device_tensor(out, torch.float32, "out", need=ids.numel() * 6)
            if t.data_ptr() != out.data_ptr():
                raise ValueError("out must be a contiguous float32 CUDA tensor")
        else:
            t = torch.empty((ids.numel(), 6), dtype=torch.float32, device=ids.device)
        _check(lib().qap_orbit_targets(self.h, C.c_void_p(ids.data_ptr()), ids.numel(),
                                       float(scale), C.c_void_p(t.data_ptr())), self.h)
        return t

    def orbit_outputs(self, mlp: "Mlp"):
        import torch

        y = torch.empty((orbit_count(self.n), 6), dtype=torch.float32, device="cuda")
        _check(lib().qap_orbit_outputs(self.h, mlp.h, C.c_void_p(y.data_ptr())), self.h)
        return y

    def warm_start_outputs(self, y, scale: float):
        """y: float32 CUDA tensor of orbit_count(n) x 6 outputs in orbit-id order."""
        import torch

        y = _device_tensor(y, torch.float32, "y", need=orbit_count(self.n) * 6)
        _check(lib().qap_warm_start_outputs(self.h, C.c_void_p(y.data_ptr()), float(scale)), self.h)

    def warm_start(self, mlp: "Mlp", gain: float | None = None):
        """Learned S-form start; gain defaults to the perceptron's own."""
        st = QapWarmStats()
        g = mlp.gain if gain is None else float(gain)
        _check(lib().qap_warm_start(self.h, mlp.h, g, C.byref(st)), self.h)
        return {"orbits": st.orbits, "scale": st.scale, "gain": st.gain, "ms_mlp": st.ms_mlp,
                "ms_write": st.ms_write, "seconds": st.seconds, "mlp_flops": st.mlp_flops}


def _device_tensor(t, dtype, name: str, need: int | None = None):
    """The learned calls hand raw device pointers to kernels: refuse, before
    any launch, a tensor that is not a CUDA tensor of the given dtype or, when
    `need` is given, does not hold exactly that many elements."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, not {t.dtype}")
    if need is not None and t.numel() != need:
        raise ValueError(f"{name} must hold {need} elements, not {t.numel()}")
    return t.contiguous()


def _samples(t, cols: int, name: str, rows: int | None = None):
    """A (rows, cols) float32 CUDA tensor of perceptron samples, checked."""
    import torch

    t = _device_tensor(t, torch.float32, name)
    if t.dim() != 2 or t.shape[1] != cols or (rows is not None and t.shape[0] != rows):
        want = f"({'count' if rows is None else rows}, {cols})"
        raise ValueError(f"{name} must have shape {want}, not {tuple(t.shape)}")
    return t


def orbit_count(n: int) -> int:
    c = C.c_int64(0)
    _check(lib().qap_orbit_count(int(n), C.byref(c)))
    return c.value


def pack_mlp_params(tensors: dict) -> np.ndarray:
    """Concatenate W1, b1, W2, b2, W3, b3 (any float arrays) into the
    library's float32 parameter block."""
    parts = []
    for name, shape in MLP_SHAPES:
        a = np.asarray(tensors[name], dtype=np.float32)
        if a.shape != shape:
            raise ValueError(f"{name}: shape {a.shape}, expected {shape}")
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unpack_mlp_params(flat) -> dict:
    out, o = {}, 0
    for name, shape in MLP_SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + k]).reshape(shape)
        o += k
    return out


class Mlp:
    """The warm start's perceptron on the GPU (float32 masters, bf16 MFMA
    kernels).  Device tensors are torch CUDA tensors."""

    def __init__(self, params, max_batch: int = 8192, stream: int | None = None, gain: float | None = None):
        import torch

        if gain is None:
            gain = float(params.get("gain", 1.0)) if isinstance(params, dict) else 1.0
        self.gain = float(gain)  # multiplier gain used by DualAscent.warm_start
        flat = params if isinstance(params, np.ndarray) and params.ndim == 1 else pack_mlp_params(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != MLP_PARAMS:
            raise ValueError("parameter block of 75782 floats expected")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        _check(lib().qap_mlp_create(flat.ctypes.data_as(C.POINTER(C.c_float)), self.max_batch,
                                    C.c_void_p(stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().qap_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream: int):
        _check(lib().qap_mlp_set_stream(self.h, C.c_void_p(stream)))

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().qap_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def forward(self, x):
        import torch

        x = _samples(x, 32, "x")
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
        _check(lib().qap_mlp_forward(self.h, C.c_void_p(x.data_ptr()), x.shape[0],
                                     C.c_void_p(y.data_ptr())))
        return y

    def gradients(self, x, t):
        x = _samples(x, 32, "x")
        t = _samples(t, 6, "t", rows=x.shape[0])
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = C.c_double(0.0)
        _check(lib().qap_mlp_gradients(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       x.shape[0], g.ctypes.data_as(C.POINTER(C.c_float)),
                                       C.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> float:
        x = _samples(x, 32, "x")
        t = _samples(t, 6, "t", rows=x.shape[0])
        opt = QapAdamParams(float(lr), float(beta1), float(beta2), float(eps))
        loss = C.c_double(0.0)
        _check(lib().qap_mlp_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                        x.shape[0], C.byref(opt), C.byref(loss)))
        return loss.value


def batch_run(handles, iters: int, window: int = 0, min_improve: float = 0.0,
              ub_cut: float = float("inf"), static: bool = False, zlap_lanes: int = 0):
    """Advance several DualAscent handles (any sizes) with the batched kernels;
    static=True calls the entry point that allocates nothing
    (qap_batch_dual_ascent_static); zlap_lanes picks the Z-LAP mapping (0:
    timed choice; 8..64 lane groups; -1, -2 one or two tiles per wavefront)."""
    arr = (C.c_void_p * len(handles))(*[hd.h.value for hd in handles])
    bp = QapBatchParams(int(iters), int(window), float(min_improve), float(ub_cut), int(zlap_lanes), 0)
    st = QapBatchStats()
    fn = lib().qap_batch_dual_ascent_static if static else lib().qap_batch_dual_ascent
    code = fn(arr, len(handles), C.byref(bp), C.byref(st))
    _check(code, handles[0].h if handles else None)
    return {"iterations": st.iterations, "stopped": st.stopped, "fathomed": st.fathomed,
            "window_stops": st.window_stops, "compactions": st.compactions, "seconds": st.seconds}


def lap_batch(cost, lanes: int = 0, cols: int = 0, stream: int | None = None):
    """Solve a batch of LAPs on the GPU.  cost: torch float64 CUDA tensor of
    shape (count, m, m).  Returns (theta, u, v, row_of_col) as tensors."""
    import torch

    if not (cost.is_cuda and cost.dtype == torch.float64 and cost.dim() == 3):
        raise ValueError("cost must be a float64 CUDA tensor (count, m, m)")
    cost = cost.contiguous()
    count, m, m2 = cost.shape
    if m != m2:
        raise ValueError("square matrices required")
    u = torch.empty((count, m), dtype=torch.float64, device=cost.device)
    v = torch.empty_like(u)
    th = torch.empty((count,), dtype=torch.float64, device=cost.device)
    rc = torch.empty((count, m), dtype=torch.int32, device=cost.device)
    if stream is None:
        stream = torch.cuda.current_stream(cost.device).cuda_stream
    code = lib().qap_lap_batch(C.c_void_p(cost.data_ptr()), count, m, C.c_void_p(u.data_ptr()),
                               C.c_void_p(v.data_ptr()), C.c_void_p(th.data_ptr()),
                               C.c_void_p(rc.data_ptr()), int(lanes), int(cols), C.c_void_p(stream))
    _check(code)
    return th, u, v, rc


# ---- layout helpers (host-side index maps of the documented layout) ------

def tile_index(n: int, i: int, p: int, j: int, q: int) -> int:
    jp = j - (j > i)
    qp = q - (q > p)
    return ((i * n + p) * (n - 1) + jp) * (n - 1) + qp


def location_automorphisms(D, B=None, cap: int = 4096) -> np.ndarray:
    """Location permutations keeping D (and B's columns): rows of the result,
    identity first (host computation in the library)."""
    D = _f64(D)
    n = D.shape[0]
    Bp = None if B is None else _f64(B)
    out = np.zeros((cap, n), dtype=np.int32)
    cnt = C.c_int(0)
    _check(lib().qap_location_automorphisms(n, _dptr(D), None if Bp is None else _dptr(Bp), int(cap),
                                            C.c_void_p(out.ctypes.data), C.byref(cnt)))
    return out[:cnt.value].copy()
