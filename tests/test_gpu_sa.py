"""GPU parity of the Type 4 ascent with simulated annealing (Section 2.3's
last rule, Section 5's schedule): the HIP library through its C ABI against
the CPU oracle with the same SplitMix64 seed.  Both sides draw the same
numbers and take the same steps, so bounds, slacks and step counts agree bit
for bit (np.array_equal)."""
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


def _pair(inst, t0_of_ub, seed, gpu_kw=None, cpu_kw=None, warm=2, **sa):
    F, D, Bm = inst.arrays()
    gpu = B.DualAscent(F, D, Bm, **(gpu_kw or {}))
    cpu = O.DualAscent(F, D, Bm, **(cpu_kw or {}))
    gpu.run(warm)
    cpu.run(warm)
    t0 = t0_of_ub * cpu.UB
    gpu.set_annealing(t0, seed=seed, **sa)
    cpu.set_annealing(t0, seed=seed, **sa)
    return gpu, cpu


@pytest.mark.parametrize("inst", [I.random_instance(8, 3), I.random_instance(9, 11),
                                  I.grid_instance(10, 2, 5, 0.4, 1, 9, 6), I.dense_instance(12, 4),
                                  I.dense_instance(17, 11)], ids=lambda x: x.name)
def test_frequent_steps_parity(inst):
    """A temperature that takes most steps (each gives away up to a quarter
    of the bound): every iteration's bound, the state after each call and
    the step count agree with the oracle."""
    n = inst.n
    gpu, cpu = _pair(inst, 10.0, seed=5)
    for chunk in (1, 4, 15):
        g = gpu.run(chunk)
        c = cpu.run(chunk)
        assert g["iterations_done"] == c
        _compare_state(gpu, cpu, n)
        assert g["sa_steps"] == cpu.sa_accepted
    tr = gpu.trace()
    assert np.array_equal(tr, cpu.trace())
    assert g["best_lb"] == tr.max()
    assert cpu.sa_accepted >= 5


def test_section5_schedule_parity_300_iterations():
    """t0 = 4 % of the incumbent, kappa_max 0.25, cooling 0.99 per 100
    iterations: a few steps in 300 iterations, taken on the same iterations
    as the oracle's; the best bound is no worse than F1's."""
    inst = I.grid_instance(10, 2, 5, 0.4, 1, 9, 6)
    F, D, Bm = inst.arrays()
    gpu, cpu = _pair(inst, 0.04, seed=1)
    g = gpu.run(298)
    cpu.run(298)
    assert np.array_equal(gpu.trace(), cpu.trace())
    _compare_state(gpu, cpu, 10)
    assert g["sa_steps"] == cpu.sa_accepted >= 1
    f1 = B.DualAscent(F, D, Bm)
    f1.run(300)
    assert g["best_lb"] >= f1.run(0)["lb"]


@pytest.mark.parametrize("variant", ["half", "f2", "mapping16"])
def test_annealing_with_other_variants(variant):
    inst = I.random_instance(9, 11)
    n = 9
    if variant == "half":
        gpu, cpu = _pair(inst, 10.0, 9, gpu_kw=dict(params=B.half_params()), cpu_kw=dict(params=O.HALF))
    elif variant == "f2":
        gpu, cpu = _pair(inst, 10.0, 9, gpu_kw=dict(two_phase=1), cpu_kw=dict(two_phase=True))
    else:
        gpu, cpu = _pair(inst, 10.0, 9, gpu_kw=dict(zlap_lanes=16))
    gpu.run(20)
    cpu.run(20)
    assert np.array_equal(gpu.trace(), cpu.trace())
    _compare_state(gpu, cpu, n)


def test_annealing_off_again_and_refusals():
    inst = I.random_instance(8, 3)
    F, D, Bm = inst.arrays()
    gpu, cpu = _pair(inst, 10.0, seed=2)
    gpu.run(5)
    cpu.run(5)
    gpu.set_annealing(0.0)
    cpu.set_annealing(0.0)
    gpu.run(5)
    cpu.run(5)
    assert np.array_equal(gpu.trace(), cpu.trace())
    _compare_state(gpu, cpu, 8)
    gpu.set_annealing(100.0)
    for call in [lambda: gpu.track(), lambda: gpu.fold(0, 0), lambda: gpu.bnb_solve(),
                 lambda: B.batch_run([gpu], 1)]:
        with pytest.raises(B.QapError) as e:
            call()
        assert e.value.code == -5
    for bad in [dict(kappa_max=2.0), dict(cool=1.5), dict(period=0)]:
        with pytest.raises(B.QapError) as e:
            gpu.set_annealing(100.0, **bad)
        assert e.value.code == -1
    tr = B.DualAscent(F, D, Bm)
    tr.track()
    with pytest.raises(B.QapError) as e:
        tr.set_annealing(100.0)
    assert e.value.code == -5


def test_annealing_full_size_n30_dense():
    """n = 30 dense, the benchmark's mapping, t0 = 4 % of the incumbent:
    every bound below the incumbent, best_lb the trace's maximum, slacks
    non-negative on sampled tiles."""
    F, D, Bm = I.dense_n30().arrays()
    h = B.DualAscent(F, D, Bm)
    r = h.run(2)
    h.set_annealing(0.04 * r["ub"], seed=3)
    g = h.run(30)
    tr = h.trace()
    assert tr.max() <= g["ub"] and g["best_lb"] == tr.max()
    assert g["lb"] <= tr[-1]
    T = 30 * 30 * 29 * 29
    got = h.export_tiles([int(t) for t in np.random.default_rng(4).integers(0, T, 32)])
    assert got.min() >= -1e-9 * F.max() * D.max()
