"""Seeded synthetic QAP instances (flows F, distances D, fixed costs B).

This module only draws numbers; it holds none of the dual-ascent arithmetic.
It is shared by the CPU oracle tests, the GPU tests and the benchmark so that
both sides read the very same instance.

The instances stand in for the QAPLIB families the paper measures on
(Section 5): Nugent-like instances place the locations on a rectangular grid
with Manhattan distances and sparse integer flows; Taillard-a-like instances
have dense uniform integer flows and distances.  No QAPLIB file is reproduced.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* grid: location p sits at cell (p // cols, p % cols); d_pq is the Manhattan
  distance between the cells.
* sparse symmetric flows: for i < j in row-major order draw
  ``zero = rng.random() < p0`` then ``val = rng.integers(lo, hi + 1)`` (both
  always drawn); f_ij = f_ji = 0 if zero else val; zero diagonal.
* dense symmetric: the upper triangle of F (i < j row-major, one
  ``rng.integers(lo, hi + 1)`` each) then the upper triangle of D the same way;
  both mirrored, zero diagonals.
* B = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Instance:
    name: str
    n: int
    F: np.ndarray  # (n, n) float64, flows
    D: np.ndarray  # (n, n) float64, distances
    B: np.ndarray  # (n, n) float64, fixed costs

    def arrays(self):
        return self.F, self.D, self.B


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_distances(n: int, rows: int, cols: int) -> np.ndarray:
    if rows * cols < n:
        raise ValueError("grid too small for n locations")
    D = np.zeros((n, n), dtype=np.float64)
    for p in range(n):
        rp, cp = divmod(p, cols)
        for q in range(n):
            rq, cq = divmod(q, cols)
            D[p, q] = abs(rp - rq) + abs(cp - cq)
    return D


def sparse_symmetric_flows(n: int, rng: np.random.Generator, p0: float,
                           lo: int, hi: int) -> np.ndarray:
    F = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(i + 1, n):
            zero = rng.random() < p0
            val = int(rng.integers(lo, hi + 1))
            v = 0.0 if zero else float(val)
            F[i, j] = v
            F[j, i] = v
    return F


def dense_symmetric(n: int, rng: np.random.Generator, lo: int, hi: int) -> np.ndarray:
    M = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(i + 1, n):
            v = float(rng.integers(lo, hi + 1))
            M[i, j] = v
            M[j, i] = v
    return M


def grid_instance(n: int, rows: int, cols: int, p0: float, lo: int, hi: int,
                  seed: int, name: str | None = None) -> Instance:
    rng = _rng(seed)
    F = sparse_symmetric_flows(n, rng, p0, lo, hi)
    D = grid_distances(n, rows, cols)
    B = np.zeros((n, n), dtype=np.float64)
    return Instance(name or f"grid{rows}x{cols}_n{n}_s{seed}", n, F, D, B)


def dense_instance(n: int, seed: int, lo: int = 0, hi: int = 99,
                   name: str | None = None) -> Instance:
    rng = _rng(seed)
    F = dense_symmetric(n, rng, lo, hi)
    D = dense_symmetric(n, rng, lo, hi)
    B = np.zeros((n, n), dtype=np.float64)
    return Instance(name or f"dense_n{n}_s{seed}", n, F, D, B)


def random_instance(n: int, seed: int, lo: int = 0, hi: int = 9,
                    asymmetric: bool = True, with_b: bool = True) -> Instance:
    """General test instance: independent integer entries (asymmetric F, D,
    nonzero diagonals and fixed costs) to exercise every term of the QAP."""
    rng = _rng(seed)
    F = rng.integers(lo, hi + 1, size=(n, n)).astype(np.float64)
    D = rng.integers(lo, hi + 1, size=(n, n)).astype(np.float64)
    if not asymmetric:
        F = np.triu(F, 1) + np.triu(F, 1).T
        D = np.triu(D, 1) + np.triu(D, 1).T
    B = (rng.integers(lo, hi + 1, size=(n, n)).astype(np.float64)
         if with_b else np.zeros((n, n)))
    return Instance(f"rand_n{n}_s{seed}", n, F, D, B)


# ---- the named workloads -------------------------------------------------

def grid_n8() -> Instance:
    """n = 8 on a 2x4 grid, flows 0 w.p. 0.4 else U{1..9}, seed 0."""
    return grid_instance(8, 2, 4, 0.4, 1, 9, 0, name="grid2x4_n8")


def grid_n15() -> Instance:
    """n = 15 on a 3x5 grid, flows 0 w.p. 0.4 else U{1..10}, seed 0."""
    return grid_instance(15, 3, 5, 0.4, 1, 10, 0, name="grid3x5_n15")


def dense_n14() -> Instance:
    """n = 14, dense symmetric F and D ~ U{0..99}, zero diagonals, seed 0."""
    return dense_instance(14, 0, name="dense_n14")


def dense_n30() -> Instance:
    """n = 30, dense symmetric F and D ~ U{0..99}, zero diagonals, seed 0."""
    return dense_instance(30, 0, name="dense_n30")


def grid_n30() -> Instance:
    """n = 30 on a 5x6 grid, flows 0 w.p. 0.4 else U{1..10}, seed 0."""
    return grid_instance(30, 5, 6, 0.4, 1, 10, 0, name="grid5x6_n30")


def dense_n42() -> Instance:
    """n = 42, dense symmetric F and D ~ U{0..99}, zero diagonals, seed 0."""
    return dense_instance(42, 0, name="dense_n42")


def learned_family(idx: int) -> Instance:
    """Instance idx of the 80-instance warm-start family: even idx are grid
    instances (rows = floor(sqrt n), cols = ceil(n / rows), flows 0 w.p. 0.4
    else U{1..10}), odd idx are dense U{0..99}; n = 20 + (idx // 2) % 11,
    seed = 1000 + idx.  idx < 64 is the training split, idx >= 64 held out."""
    n = 20 + (idx // 2) % 11
    seed = 1000 + idx
    if idx % 2 == 0:
        rows = int(math.isqrt(n))
        cols = -(-n // rows)
        return grid_instance(n, rows, cols, 0.4, 1, 10, seed, name=f"fam{idx}_grid_n{n}")
    return dense_instance(n, seed, name=f"fam{idx}_dense_n{n}")


NAMED = {
    "grid_n8": grid_n8,
    "grid_n15": grid_n15,
    "dense_n14": dense_n14,
    "dense_n30": dense_n30,
    "grid_n30": grid_n30,
    "dense_n42": dense_n42,
}


def named(name: str) -> Instance:
    return NAMED[name]()
