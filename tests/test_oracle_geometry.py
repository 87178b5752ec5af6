"""Pins for oracle.geometry: counting identities, the paper's hexagonal-array
numbers, the degeneracy criterion and a hand-worked selection."""
import math
import os

import numpy as np
import pytest

from oracle import geometry as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7])
def test_square_types_equal_bruteforce(n):
    pos = G.square_positions(n)
    t_bf, groups = G.baseline_types(pos)
    t_cf, sizes = G.square_types(n)
    assert t_bf == t_cf
    assert [len(g) for g in groups] == sizes
    # pair orientation r_i - r_j = d for every pair of every group
    for d, grp in zip(t_bf, groups):
        for i, j in grp:
            assert tuple(pos[i] - pos[j]) == d


@pytest.mark.parametrize("n", [2, 3, 8, 16, 33])
def test_group_counting_identities(n):
    types, sizes = G.square_types(n)
    nant = n * n
    assert sum(sizes) == nant * (nant - 1) // 2       # every unordered pair exactly once
    assert len(types) == 2 * n * (n - 1)               # canonical half-plane of (2n-1)^2 - 1 lags


@pytest.mark.parametrize("n", [3, 6])
def test_group_pairs_matches_bruteforce(n):
    pos = G.square_positions(n)
    types, groups = G.baseline_types(pos)
    pairs, tix = G.group_pairs(pos, types)
    flat = [p for g in groups for p in g]
    assert [tuple(p) for p in pairs] == flat
    assert list(tix) == [t for t, g in enumerate(groups) for _ in g]


def test_hex_array_counts_from_paper():
    # Fig. 2 / Sec. 5: the three shortest baseline-types of the prototype hex
    # array have 30 redundant pairs each.
    pos = G.hex_positions(4)
    assert len(pos) == 37
    types, groups = G.baseline_types(pos, G.HEX_METRIC)
    assert [len(g) for g in groups[:3]] == [30, 30, 30]
    # Sec. 5.4: with the three shortest types, a corner antenna takes part in
    # three measurements, an edge antenna in four and a central one in six.
    deg = np.zeros(len(pos), dtype=int)
    for grp in groups[:3]:
        for i, j in grp:
            deg[i] += 1
            deg[j] += 1
    r = 3
    a, b = pos[:, 0], pos[:, 1]
    ring = np.maximum.reduce([np.abs(a), np.abs(b), np.abs(a + b)])
    nmax = (np.abs(a) == r).astype(int) + (np.abs(b) == r).astype(int) + (np.abs(a + b) == r).astype(int)
    corner = (ring == r) & (nmax >= 2)
    edge = (ring == r) & ~corner
    assert corner.sum() == 6
    assert set(deg[corner]) == {3}
    assert set(deg[edge]) == {4}
    assert set(deg[ring < r]) == {6}
    # Sec. 6.4 studies a 331-antenna array: the hex number of side 11.
    assert len(G.hex_positions(11)) == 331


def test_degeneracy_criterion():
    # Sec. 5.2: the null space must hold exactly the four degeneracies.
    sq = G.square_positions(6)
    # bipartite nearest-neighbour graph: an extra checkerboard amplitude mode
    assert G.nullity(sq, [(1, 0), (0, 1)]) == (2, 3)
    assert G.nullity(sq, [(1, 0), (0, 1), (-1, 1)]) == (1, 3)
    assert G.nullity(sq, G.square_types(6)[0][:7]) == (1, 3)
    # hexagonal layout: three shortest types are the minimum (Sec. 5.2)
    hx = G.hex_positions(4)
    types, _ = G.baseline_types(hx, G.HEX_METRIC)
    assert sum(G.nullity(hx, types[:3])) == 4
    assert sum(G.nullity(hx, types[:2])) > 4


def test_checkerboard_null_vector_explicit():
    n = 5
    pos = G.square_positions(n)
    pairs, tix = G.group_pairs(pos, [(1, 0), (0, 1)])
    a = (-1.0) ** (pos[:, 0] + pos[:, 1])
    assert np.all(a[pairs[:, 0]] + a[pairs[:, 1]] == 0)


def test_selection_hand_worked():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "selection_n8.txt")) if l.strip() and not l.startswith("#")]
    pos = G.square_positions(8)
    for base, k, npairs in rows:
        lb = math.e if base == "e" else float(base)
        sel = G.select_subset_square(8, 1.0, lb)
        pairs, _ = G.group_pairs(pos, sel)
        assert len(sel) == int(k)
        assert len(pairs) == int(npairs)
        assert G.select_subset(pos, G.SQUARE_METRIC, 1.0, lb) == sel


def test_selection_budget_closest_prefix():
    # closest whole-group prefix for several grids, checked against the budget
    for n in [8, 12, 16, 24]:
        types, sizes = G.square_types(n)
        cum = np.cumsum(sizes)
        b = G.subset_budget(n * n)
        sel = G.select_subset_square(n)
        k = len(sel)
        assert abs(cum[k - 1] - b) <= abs(cum[k] - b)
        if k >= 2:
            assert abs(cum[k - 1] - b) <= abs(cum[k - 2] - b)


def test_hex_grid_lays_the_hexagon_on_its_lattice_grid():
    # Sec. 3 / Fig. 2 layout in lattice coordinates: the side-4 hexagon fits
    # a 7 x 7 index grid, 37 of whose 49 points are antennas
    n, mask, pos = G.hex_grid(4)
    assert n == 7 and mask.sum() == 37 and len(pos) == 37
    assert np.array_equal(pos, G.hex_positions(4) + 3)
    assert pos.min() == 0 and pos.max() == 6
    # raster order (y major, x minor) and the mask agree
    assert np.array_equal(np.nonzero(mask)[0], pos[:, 1] * n + pos[:, 0])
    # the 30 pairs of each nearest-neighbour direction survive the shift
    for d in [(1, 0), (0, 1), (-1, 1)]:
        assert len(G.PositionIndex(pos).pairs_of(*d)[0]) == 30
