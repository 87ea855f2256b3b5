"""The C ABI library loads and exports every symbol include/qap_rlt2.h
declares; argument validation that needs no device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1710_03732_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "qap_rlt2.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qap_[a-z0-9_]+)\s*\(", src)) -
                  {"qap_alloc_fn", "qap_free_fn"})


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(B.EXPORTED) == set(names)


def test_version_and_defaults():
    assert "gfx950" in B.version()
    p = B.default_params()
    assert p.kappa_z == 5.0 / 6.0 and p.kappa_y == 1.0 and p.kappa_x == 1.0
    assert p.phi_z == 0.2 and p.phi_y == 0.5


def test_workspace_bytes():
    assert B.workspace_bytes(2) == 0 and B.workspace_bytes(65) == 0
    w30 = B.workspace_bytes(30)
    V = (30 * 29 * 28) ** 2
    assert 8 * V < w30 < 8 * V * 1.1
    assert B.workspace_bytes(42) < 288e9


@pytest.mark.parametrize("n,code", [(2, -5), (65, -5)])
def test_init_rejects_unsupported_n(n, code):
    F = np.zeros((n, n))
    with pytest.raises(B.QapError) as e:
        B.DualAscent(F, F)
    assert e.value.code == code


def test_init_rejects_non_finite():
    F = np.ones((5, 5))
    F[1, 2] = np.nan
    with pytest.raises(B.QapError) as e:
        B.DualAscent(F, np.ones((5, 5)))
    assert e.value.code == -1


def test_init_rejects_bad_params():
    F = np.ones((5, 5))
    with pytest.raises(B.QapError) as e:
        B.DualAscent(F, F, kappa_z=1.5)
    assert e.value.code == -1
    with pytest.raises(B.QapError) as e:
        B.DualAscent(F, F, phi_z=0.3)
    assert e.value.code == -1


def test_half_parameters_are_validated_before_any_device_call():
    """HALF needs phi_z = 1/2 (two upper partners) and the scalar Z-LAP
    mapping; an unknown scheme or field is refused."""
    F = np.ones((5, 5))
    p = B.half_params()
    assert (p.kappa_z, p.kappa_y, p.kappa_x, p.phi_z, p.phi_y) == (2.0 / 3.0, 1.0, 1.0, 0.5, 0.5)
    assert p.scheme == B.SCHEME_HALF and p.zlap_lanes == -1
    for bad in [dict(phi_z=0.2), dict(zlap_lanes=16, zlap_cols=2), dict(scheme=2)]:
        with pytest.raises(B.QapError) as e:
            B.DualAscent(F, F, params=B.half_params(**bad))
        assert e.value.code == -1, bad
    with pytest.raises(B.QapError) as e:
        B.DualAscent(F, F, phi_z=0.5)  # FULL with the HALF share
    assert e.value.code == -1
    with pytest.raises(TypeError):
        B.default_params(shceme=1)
    for bad in [B.half_params(two_phase=1), B.default_params(two_phase=2)]:
        with pytest.raises(B.QapError) as e:  # F2 is FULL-only; 0/1 only
            B.DualAscent(F, F, params=bad)
        assert e.value.code == -1


def test_lap_batch_rejects_bad_sizes():
    lib = B.lib()
    assert lib.qap_lap_batch(None, 1, 0, None, None, None, None, 0, 0, None) == -1
    assert lib.qap_lap_batch(None, 1, 1025, None, None, None, None, 0, 0, None) == -1
    assert lib.qap_lap_batch(None, 1, 65, None, None, None, None, 0, 0, None) == -1  # NULL pointers
    assert lib.qap_lap_batch(None, 0, 5, None, None, None, None, 0, 0, None) == 0


def test_orbit_count_and_learned_entry_points_validate():
    lib = B.lib()
    c = ctypes.c_int64(0)
    assert lib.qap_orbit_count(3, ctypes.byref(c)) == 0 and c.value == 6
    assert lib.qap_orbit_count(30, ctypes.byref(c)) == 0 and c.value == 4060 * 24360
    assert lib.qap_orbit_count(2, ctypes.byref(c)) == -1
    assert lib.qap_orbit_count(65, ctypes.byref(c)) == -1
    assert lib.qap_track(None, 1) == -1
    assert lib.qap_get_multipliers(None, None, None) == -1
    assert lib.qap_set_multipliers(None, None, None) == -1
    assert lib.qap_warm_start_outputs(None, None, 1.0) == -1
    assert lib.qap_warm_start(None, None, 1.0, None) == -1
    out = ctypes.c_void_p()
    assert lib.qap_mlp_create(None, 16, None, ctypes.byref(out)) == -1
    params = np.zeros(B.MLP_PARAMS, dtype=np.float32)
    fp = params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert lib.qap_mlp_create(fp, 0, None, ctypes.byref(out)) == -1
    params[7] = np.nan
    assert lib.qap_mlp_create(fp, 16, None, ctypes.byref(out)) == -1
    assert lib.qap_mlp_destroy(None) == -1


def test_mlp_parameter_packing_round_trip():
    rng = np.random.default_rng(0)
    p = {name: rng.standard_normal(shape) for name, shape in B.MLP_SHAPES}
    flat = B.pack_mlp_params(p)
    assert flat.dtype == np.float32 and flat.size == B.MLP_PARAMS
    back = B.unpack_mlp_params(flat)
    for name, _ in B.MLP_SHAPES:
        np.testing.assert_array_equal(back[name], p[name].astype(np.float32))


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the HIP library every entry point raises."""
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libqaprlt2.so")
    with pytest.raises(RuntimeError, match="HIP library missing"):
        B.lib()
    with pytest.raises(RuntimeError):
        B.DualAscent(np.ones((5, 5)), np.ones((5, 5)))


def test_learned_calls_refuse_bad_tensors_before_any_launch():
    """The learned calls pass raw device pointers to kernels, so the binding
    refuses host tensors, wrong dtypes and wrong sizes with ValueError before
    the library is called (the handles here are never created on a device)."""
    import torch

    da = B.DualAscent.__new__(B.DualAscent)  # no device state: validation comes first
    da.h, da.n, da.m, da.T = None, 8, 6, B.tile_count(8)
    ids_cpu = torch.arange(10, dtype=torch.int64)
    with pytest.raises(ValueError, match="CUDA"):
        da.orbit_features(ids_cpu)
    with pytest.raises(ValueError, match="CUDA"):
        da.orbit_targets(ids_cpu, 1.0)
    y = torch.zeros((B.orbit_count(8), 6), dtype=torch.float32)
    with pytest.raises(ValueError, match="CUDA"):
        da.warm_start_outputs(y, 1.0)
    mlp = B.Mlp.__new__(B.Mlp)
    mlp.h = None
    x = torch.zeros((4, 32), dtype=torch.float32)
    with pytest.raises(ValueError, match="CUDA"):
        mlp.forward(x)
    with pytest.raises(ValueError, match="CUDA"):
        mlp.gradients(x, torch.zeros((4, 6)))
    with pytest.raises(ValueError, match="CUDA"):
        mlp.train_step(x, torch.zeros((4, 6)))
    with pytest.raises(ValueError):
        da.orbit_features([1, 2, 3])


def test_tensor_checks_of_the_learned_calls():
    """dtype, element-count and shape rules of the checks themselves, on
    tensors that claim to be on a device (is_cuda patched): int32 ids, a
    short or float64 y, samples with the wrong width or row count."""
    import torch

    class Fake(torch.Tensor):
        @property
        def is_cuda(self):
            return True

    def fake(t):
        return t.as_subclass(Fake)

    B._device_tensor(fake(torch.zeros(5, dtype=torch.int64)), torch.int64, "ids")
    with pytest.raises(ValueError, match="dtype"):
        B._device_tensor(fake(torch.zeros(5, dtype=torch.int32)), torch.int64, "ids")
    with pytest.raises(ValueError, match="elements"):
        B._device_tensor(fake(torch.zeros((3, 6), dtype=torch.float32)), torch.float32, "y", need=24)
    with pytest.raises(ValueError, match="dtype"):
        B._device_tensor(fake(torch.zeros((4, 6), dtype=torch.float64)), torch.float32, "y", need=24)
    B._samples(fake(torch.zeros((4, 32), dtype=torch.float32)), 32, "x")
    with pytest.raises(ValueError, match="shape"):
        B._samples(fake(torch.zeros((4, 31), dtype=torch.float32)), 32, "x")
    with pytest.raises(ValueError, match="shape"):
        B._samples(fake(torch.zeros((5, 6), dtype=torch.float32)), 6, "t", rows=4)
