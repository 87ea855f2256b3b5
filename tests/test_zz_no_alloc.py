"""The batched dual ascent that allocates nothing (qap_batch_dual_ascent_static)
against the allocating one, through the C ABI: two calls in a row, the
second on fewer and smaller handles, every handle's bound trace and state
bitwise equal; the static workspace's limits are refused before any device
work."""
import numpy as np
import pytest

from paper_1710_03732_amd import binding as B
from paper_1710_03732_amd import instances as I

pytestmark = pytest.mark.gpu


def _handles():
    """Fresh roots of sizes 4..12 and three folded children of a 10-node
    parent (sizes 9), built the same way each call."""
    out = []
    for inst in (I.random_instance(4, 160), I.dense_instance(12, 161), I.grid_instance(9, 3, 3, 0.4, 1, 10, 162),
                 I.random_instance(6, 163, lo=-2, hi=6)):
        F, D, Bm = inst.arrays()
        out.append(B.DualAscent(F, D, Bm))
    F, D, Bm = I.dense_instance(10, 164).arrays()
    par = B.DualAscent(F, D, Bm)
    par.run(2)
    for (l, s) in [(0, 1), (4, 4), (9, 0)]:
        out.append(par.fold(l, s))
    return out


def _same(a, b):
    assert np.array_equal(a.trace(), b.trace()), (a.n, a.trace(), b.trace())
    ha, xa, ya, za = a.export_state()
    hb, xb, yb, zb = b.export_state()
    assert (ha.t, ha.lb, ha.ub, ha.checksum) == (hb.t, hb.lb, hb.ub, hb.checksum)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(za, zb)


def test_static_batch_equals_allocating_batch_twice():
    ref, sta = _handles(), _handles()
    s1 = B.batch_run(ref, iters=12)
    s2 = B.batch_run(sta, iters=12, static=True)
    assert s1["iterations"] == s2["iterations"] and s1["stopped"] == s2["stopped"]
    for a, b in zip(ref, sta):
        _same(a, b)
    # second call: fewer handles, the smallest ones (the workspace keeps the
    # first call's tables; this call rewrites what it uses)
    small_r = [h for h in ref if h.n <= 9][:3]
    small_s = [h for h in sta if h.n <= 9][:3]
    assert len(small_r) == 3 and max(h.n for h in small_r) < max(h.n for h in ref)
    B.batch_run(small_r, iters=5)
    B.batch_run(small_s, iters=5, static=True)
    for a, b in zip(small_r, small_s):
        _same(a, b)
    for h in ref + sta:
        h.close()


def test_static_batch_refuses_beyond_its_limits():
    F, D, Bm = I.dense_instance(6, 165).arrays()
    h = B.DualAscent(F, D, Bm)
    with pytest.raises(B.QapError) as e:
        B.batch_run([h] * 257, iters=1, static=True)
    assert e.value.code == -1
    # the bound trace (1024 entries) is not grown without allocating
    with pytest.raises(B.QapError) as e:
        B.batch_run([h], iters=2000, static=True)
    assert e.value.code == -4
    st = h.status()
    assert st["t"] == 0
    h.close()
