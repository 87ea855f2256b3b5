"""Test-side maps between the oracle's dense arrays and the library's compact
layout (documented in include/qap_rlt2.h).  Pure index bookkeeping."""
import numpy as np


def tile_coords(n):
    """Arrays (i, p, j, q) for every tile index t in order."""
    m1 = n - 1
    t = np.arange(n * n * m1 * m1)
    qp = t % m1
    jp = (t // m1) % m1
    ip = t // (m1 * m1)
    i, p = ip // n, ip % n
    j = jp + (jp >= i)
    q = qp + (qp >= p)
    return i, p, j, q


def tile_index(n, i, p, j, q):
    jp = j - (j > i)
    qp = q - (q > p)
    return ((i * n + p) * (n - 1) + jp) * (n - 1) + qp


def dense_to_compact_y(n, Y):
    i, p, j, q = tile_coords(n)
    return Y[i, j, p, q]


def dense_to_compact_z(n, Z):
    """(T, m, m) view of the dense z array in tile-major compact order."""
    m = n - 2
    i, p, j, q = tile_coords(n)
    T = len(i)
    kk = np.arange(m)
    # row k'' -> k skipping i and j; column r'' -> r skipping p and q
    lo_f = np.minimum(i, j)[:, None]
    hi_f = np.maximum(i, j)[:, None]
    k = kk[None, :] + 0
    k = k + (k >= lo_f)
    k = k + (k >= hi_f)
    lo_l = np.minimum(p, q)[:, None]
    hi_l = np.maximum(p, q)[:, None]
    r = kk[None, :] + 0
    r = r + (r >= lo_l)
    r = r + (r >= hi_l)
    out = Z[i[:, None, None], j[:, None, None], k[:, :, None], p[:, None, None], q[:, None, None],
            r[:, None, :]]
    return out.reshape(T, m, m)
