"""Location automorphisms for the symmetry elimination of Section 4 (host
code of the library, no device work): checked against brute force over all
location permutations on small instances."""
import itertools

import numpy as np
import pytest

from paper_1710_03732_amd import binding as B
from paper_1710_03732_amd import instances as I


def _brute(D, Bm):
    n = D.shape[0]
    out = []
    for s in itertools.permutations(range(n)):
        s = np.array(s)
        if np.array_equal(D[np.ix_(s, s)], D) and np.array_equal(Bm[:, s], Bm):
            out.append(tuple(s))
    return sorted(out)


@pytest.mark.parametrize("D,Bm,size", [
    (I.grid_distances(8, 2, 4), np.zeros((8, 8)), 4),      # rectangle: flips and half turn
    (I.grid_distances(4, 2, 2), np.zeros((4, 4)), 8),      # square: the dihedral group
    (I.grid_distances(6, 2, 3), np.zeros((6, 6)), 4),
    (I.grid_distances(7, 2, 4), np.zeros((7, 7)), 1),      # an incomplete grid
    (I.grid_distances(5, 1, 5), np.zeros((5, 5)), 2),      # a line: its reversal
    (np.ones((5, 5)) - np.eye(5), np.zeros((5, 5)), 120),  # all distances equal: every permutation
])
def test_automorphisms_match_brute_force(D, Bm, size):
    got = B.location_automorphisms(D, Bm)
    assert tuple(got[0]) == tuple(range(D.shape[0]))  # identity first
    assert sorted(map(tuple, got)) == _brute(D, Bm)
    assert len(got) == size


def test_fixed_costs_and_asymmetry_break_symmetry():
    D = I.grid_distances(8, 2, 4)
    Bm = np.zeros((8, 8))
    Bm[2, 0] = 5.0  # corner 0 now differs from the other corners: no symmetry of the rectangle keeps it
    got = B.location_automorphisms(D, Bm)
    assert sorted(map(tuple, got)) == _brute(D, Bm)
    assert len(got) == 1
    Bm[2, 7] = 5.0  # ... unless the opposite corner costs the same: the half turn returns
    got = B.location_automorphisms(D, Bm)
    assert sorted(map(tuple, got)) == _brute(D, Bm)
    assert len(got) == 2
    rng = np.random.default_rng(3)
    Dr = rng.integers(0, 9, size=(7, 7)).astype(float)
    assert len(B.location_automorphisms(Dr)) == 1


def test_cap_returns_exact_automorphisms():
    D = np.ones((7, 7)) - np.eye(7)
    got = B.location_automorphisms(D, cap=50)
    assert len(got) == 50
    for s in got:
        assert np.array_equal(D[np.ix_(s, s)], D)
