"""Host emulation of the ascent sweep's launch geometry (kernels.hpp,
k_sweep<CB, ...>: block -> facility triple and location cube, thread ->
orbit, member -> z address in the compact tile layout).  For both cube
edges the kernel uses (8 and 10) and sizes with ragged cubes, every z entry
of an orbit must be addressed exactly once per sweep and inside the array;
a mistake in the index arithmetic would either skip entries or write out of
bounds.  Pure index bookkeeping: no device and no oracle."""
import numpy as np
import pytest


def _cover(n, cb):
    m = n - 2
    mm = m * m
    T = n * n * (n - 1) * (n - 1)
    tris = [(i, j, k) for i in range(n) for j in range(i + 1, n) for k in range(j + 1, n)]
    nb = (n + cb - 1) // cb
    nb3 = nb ** 3
    blocks = (len(tris) + 7) // 8 * 8 * nb3
    orb = cb ** 3
    nt = (orb + 63) // 64 * 64
    tid = np.arange(nt)
    live = tid < orb
    a = [tid // (cb * cb), (tid // cb) % cb, tid % cb]
    X1, X2, X3 = [0, 0, 1, 1, 2, 2], [1, 2, 0, 2, 0, 1], [2, 1, 2, 0, 1, 0]
    cover = np.zeros(T * mm, dtype=np.int32)
    for b in range(blocks):
        xcd, s = b & 7, b >> 3
        tri = (s // nb3) * 8 + xcd
        if tri >= len(tris):
            continue
        sub = s % nb3
        base = [(sub // (nb * nb)) * cb, ((sub // nb) % nb) * cb, (sub % nb) * cb]
        fi, fj, fk = tris[tri]
        F = [(fi, fj, fk), (fi, fk, fj), (fj, fi, fk), (fj, fk, fi), (fk, fi, fj), (fk, fj, fi)]
        for e in range(6):
            loc = [None] * 3
            loc[X1[e]] = base[X1[e]] + a[0]
            loc[X2[e]] = base[X2[e]] + a[1]
            loc[X3[e]] = base[X3[e]] + a[2]
            l1, l2, l3 = loc[X1[e]], loc[X2[e]], loc[X3[e]]
            ok = live & (l1 < n) & (l2 < n) & (l3 < n) & (l1 != l2) & (l1 != l3) & (l2 != l3)
            f1, f2, f3 = F[e]
            f2p = f2 - (f2 > f1)
            row = f3 - (f3 > f1) - (f3 > f2)
            zrow = ((f1 * n + l1) * (n - 1) + f2p) * (n - 1) * mm + row * m
            l2p = l2 - (l2 > l1)
            col = l3 - (l3 > l1) - (l3 > l2)
            za = (zrow + l2p * mm + col)[ok]
            assert za.size == 0 or (za.min() >= 0 and za.max() < T * mm)
            np.add.at(cover, za, 1)
    return cover, n * (n - 1) * (n - 2) * n * (n - 1) * (n - 2)


@pytest.mark.parametrize("cb", [8, 10])
@pytest.mark.parametrize("n", [3, 4, 7, 9, 10, 11, 13, 17])
def test_every_orbit_member_addressed_once(n, cb):
    cover, members = _cover(n, cb)
    assert cover.max() == 1
    assert int(cover.sum()) == members  # all z entries with distinct facilities and locations
