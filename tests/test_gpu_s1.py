"""GPU parity of the slow variants (Section 3.4): S1, where the z
multipliers move by F1's sweep rule and every iteration solves the LAPs on
the full costs, and S2, S1 with the two-phase pooling (which then moves the
multipliers too).
The HIP library through its C ABI against the CPU oracle's S1, bit for bit
(np.array_equal): bounds, the rebuilt cost arrays and the multipliers."""
import numpy as np
import pytest

from layout import dense_to_compact_y, dense_to_compact_z
from oracle import oracle as O
from paper_1710_03732_amd import binding as B
from paper_1710_03732_amd import instances as I

pytestmark = pytest.mark.gpu


def _compare_state(gpu, cpu, n):
    hdr, x, y, z = gpu.export_state()
    X, Y, Z = cpu.export()
    assert hdr.t == cpu.t
    assert hdr.lb == cpu.LB, (hdr.lb, cpu.LB)
    assert hdr.ub == cpu.UB
    assert np.array_equal(x, X.reshape(-1))
    assert np.array_equal(y, dense_to_compact_y(n, Y))
    assert np.array_equal(z.reshape(-1, n - 2, n - 2), dense_to_compact_z(n, Z))
    v, u = gpu.multipliers()
    V, U = cpu.multipliers()
    assert np.array_equal(v.reshape(-1, n - 2, n - 2), dense_to_compact_z(n, V))
    assert not u.any() and not U.any()


def test_s1_grid_n8_iteration_by_iteration():
    F, D, Bm = I.grid_n8().arrays()
    gpu = B.DualAscent(F, D, Bm, slow=1)
    cpu = O.DualAscent(F, D, Bm, slow=True)
    for _ in range(30):
        g = gpu.run(1)
        c = cpu.run(1)
        assert g["iterations_done"] == c
        _compare_state(gpu, cpu, 8)
        if c == 0:
            break
    assert np.array_equal(gpu.trace(), cpu.trace())


@pytest.mark.parametrize("inst", [
    I.random_instance(3, 1), I.random_instance(4, 2), I.random_instance(5, 3, lo=-5, hi=5),
    I.dense_instance(9, 5), I.grid_instance(10, 2, 5, 0.4, 1, 9, 6),
    I.random_instance(12, 7, lo=0, hi=50), I.dense_instance(17, 11),
], ids=lambda x: x.name)
def test_s1_instances_parity(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    gpu = B.DualAscent(F, D, Bm, slow=1)
    cpu = O.DualAscent(F, D, Bm, slow=True)
    iters = 20 if n < 15 else 6
    g = gpu.run(iters)
    c = cpu.run(iters)
    assert g["iterations_done"] == c
    assert np.array_equal(gpu.trace(), cpu.trace())
    _compare_state(gpu, cpu, n)


@pytest.mark.parametrize("lanes,cols", [(-2, 1), (16, 1)])
def test_s1_mapping_does_not_change_results(lanes, cols):
    F, D, Bm = I.random_instance(11, 5).arrays()
    a = B.DualAscent(F, D, Bm, slow=1, zlap_lanes=-1)
    b = B.DualAscent(F, D, Bm, slow=1, zlap_lanes=lanes, zlap_cols=cols)
    a.run(10)
    b.run(10)
    assert np.array_equal(a.trace(), b.trace())


def test_s1_refusals():
    import torch
    F, D, Bm = I.random_instance(6, 9).arrays()
    h = B.DualAscent(F, D, Bm, slow=1)
    h.run(3)
    hdr, x, y, z = h.export_state()
    for call in [lambda: h.track(False), lambda: h.fold(0, 0), lambda: h.bnb_solve(),
                 lambda: B.batch_run([h], 1), lambda: h.set_annealing(100.0),
                 lambda: h.set_multipliers(np.zeros(h.T * h.m * h.m)),
                 lambda: h.import_state(hdr, x, y, z),
                 lambda: h.warm_start_outputs(torch.zeros(6 * B.orbit_count(6), device="cuda"), 1.0)]:
        with pytest.raises(B.QapError) as e:
            call()
        assert e.value.code == -5
    h.run(1)
    v0, _ = h.multipliers()
    h.track(True)  # a no-op on an S1 handle: its multipliers are its state
    assert np.array_equal(h.multipliers()[0], v0)
    for bad in [B.half_params(slow=1)]:
        with pytest.raises(B.QapError) as e:
            B.DualAscent(F, D, Bm, params=bad)
        assert e.value.code == -1


def test_s1_full_size_n30_dense():
    """n = 30 dense: iteration 0 as F1's, then bounds that never fall (to
    rounding), below the incumbent, non-negative slacks on sampled tiles."""
    F, D, Bm = I.dense_n30().arrays()
    f1 = B.DualAscent(F, D, Bm)
    s1 = B.DualAscent(F, D, Bm, slow=1)
    assert f1.run(1)["lb"] == s1.run(1)["lb"]
    g = s1.run(8)
    tr = s1.trace()
    assert np.all(np.diff(tr) >= -1e-9 * abs(tr[-1])) and tr[-1] <= g["ub"]
    T = 30 * 30 * 29 * 29
    got = s1.export_tiles([int(t) for t in np.random.default_rng(8).integers(0, T, 32)])
    assert got.min() >= -1e-9 * F.max() * D.max()


@pytest.mark.parametrize("inst", [I.grid_n8(), I.random_instance(5, 3, lo=-5, hi=5), I.dense_instance(9, 5),
                                  I.random_instance(12, 7, lo=0, hi=50), I.dense_instance(17, 11)],
                         ids=lambda x: x.name)
def test_s2_parity(inst):
    F, D, Bm = inst.arrays()
    n = inst.n
    gpu = B.DualAscent(F, D, Bm, slow=1, two_phase=1)
    cpu = O.DualAscent(F, D, Bm, slow=True, two_phase=True)
    for chunk in ((1, 1, 2, 8) if n < 15 else (1, 4)):
        g = gpu.run(chunk)
        c = cpu.run(chunk)
        assert g["iterations_done"] == c
        _compare_state(gpu, cpu, n)
    assert np.array_equal(gpu.trace(), cpu.trace())
