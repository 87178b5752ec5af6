"""Array geometry, redundant baseline groups and the subset selection rule.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Positions are integer lattice coordinates.  A square grid uses the basis
(1, 0), (0, 1); a hexagonal array (Fig. 2, Sec. 3) uses (1, 0), (1/2, sqrt3/2),
so physical lengths come from the metric G (|d|^2 = d^T G d).

A baseline-type is a displacement vector d = r_i - r_j shared by a redundant
group of antenna pairs (Sec. 2, eq. redcal: d_alpha = r_0 - r_1 for V_01).
Each unordered pair is stored once, oriented so that d lies in the canonical
half-plane (d_y > 0, or d_y = 0 and d_x > 0).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

SQUARE_METRIC = np.eye(2)
HEX_METRIC = np.array([[1.0, 0.5], [0.5, 1.0]])


def square_positions(n: int) -> np.ndarray:
    """Antenna i at (i mod n, i div n): shape [n*n, 2] int."""
    i = np.arange(n * n)
    return np.stack([i % n, i // n], axis=1)


def hex_positions(side: int) -> np.ndarray:
    """Hexagonal array with `side` antennas per edge, in axial lattice coords.

    Antennas are the lattice points (a, b) with |a|, |b|, |a + b| < side,
    listed in raster order (b major, a minor).
    """
    pts = []
    r = side - 1
    for b in range(-r, r + 1):
        for a in range(-r, r + 1):
            if abs(a + b) <= r:
                pts.append((a, b))
    return np.array(pts, dtype=np.int64)


def hex_grid(side: int):
    """A hexagonal array laid on its bounding lattice grid.

    In lattice coordinates the hexagon of `side` antennas per edge fits an
    n x n index grid, n = 2 side - 1, with (x, y) = (a + side - 1,
    b + side - 1).  Returns (n, mask, pos): mask [n*n] bool marks the
    antennas (raster index y n + x), pos [N, 2] their (x, y) in raster
    order, i.e. `hex_positions(side)` shifted onto the grid.
    """
    n = 2 * side - 1
    pos = hex_positions(side) + (side - 1)
    mask = np.zeros(n * n, dtype=bool)
    mask[pos[:, 1] * n + pos[:, 0]] = True
    return n, mask, pos


def is_canonical(dx: int, dy: int) -> bool:
    return dy > 0 or (dy == 0 and dx > 0)


def baseline_types(pos: np.ndarray, metric: np.ndarray = SQUARE_METRIC):
    """All baseline-types of an array, by brute force over antenna pairs.

    Returns (types, groups): `types` is a list of (dx, dy) sorted by
    (|d|^2, dy, dx); `groups[t]` is the list of pairs (i, j) with
    r_i - r_j = types[t], sorted by i.
    """
    groups: Dict[Tuple[int, int], List[Tuple[int, int]]] = {}
    npos = len(pos)
    for i in range(npos):
        for j in range(npos):
            if i == j:
                continue
            dx = int(pos[i, 0] - pos[j, 0])
            dy = int(pos[i, 1] - pos[j, 1])
            if is_canonical(dx, dy):
                groups.setdefault((dx, dy), []).append((i, j))

    def key(d):
        v = np.array(d, dtype=float)
        return (round(float(v @ metric @ v), 9), d[1], d[0])

    types = sorted(groups, key=key)
    return types, [sorted(groups[t]) for t in types]


def square_types(n: int):
    """Baseline-types of an n x n unit grid, without visiting pairs.

    Every canonical d with |dx|, |dy| < n occurs, with group size
    N_d = (n - |dx|)(n - |dy|).  Sorted like `baseline_types`.
    Returns (types, sizes).
    """
    types = [(dx, dy) for dy in range(0, n) for dx in range(-(n - 1), n) if is_canonical(dx, dy)]
    types.sort(key=lambda d: (d[0] * d[0] + d[1] * d[1], d[1], d[0]))
    sizes = [(n - abs(dx)) * (n - abs(dy)) for dx, dy in types]
    return types, sizes


def select_subset_square(n: int, p: float = 1.0, log_base: float = math.e):
    """`select_subset` for an n x n grid, using `square_types`."""
    pos = square_positions(n)
    types, sizes = square_types(n)
    budget = subset_budget(n * n, p, log_base)
    cum = np.cumsum(sizes)
    k = int(np.argmin(np.abs(cum - budget))) + 1
    while k <= len(types) and sum(nullity(pos, types[:k])) != 4:
        k += 1
    return types[:k]


class PositionIndex:
    """Lookup table from integer position to antenna index (-1 if empty)."""

    def __init__(self, pos: np.ndarray):
        self.pos = np.asarray(pos, dtype=np.int64)
        self.lo = self.pos.min(axis=0)
        hi = self.pos.max(axis=0)
        shape = hi - self.lo + 1
        self.lut = -np.ones((int(shape[0]), int(shape[1])), dtype=np.int64)
        self.lut[self.pos[:, 0] - self.lo[0], self.pos[:, 1] - self.lo[1]] = np.arange(len(self.pos))

    def pairs_of(self, dx: int, dy: int):
        """(i, j) index arrays of all pairs with r_i - r_j = (dx, dy), i ascending."""
        q = self.pos - np.array([dx, dy]) - self.lo
        ok = (q[:, 0] >= 0) & (q[:, 0] < self.lut.shape[0]) & (q[:, 1] >= 0) & (q[:, 1] < self.lut.shape[1])
        i = np.nonzero(ok)[0]
        j = self.lut[q[ok, 0], q[ok, 1]]
        keep = j >= 0
        return i[keep], j[keep]


def group_pairs(pos: np.ndarray, types: Sequence[Tuple[int, int]]):
    """Pairs (i, j) with r_i - r_j = d for each d in `types` (sorted by i).

    Returns (pairs [P, 2] int, tix [P] int: index of each pair's type).
    """
    idx = PositionIndex(pos)
    pi, pj, pt = [], [], []
    for t, (dx, dy) in enumerate(types):
        i, j = idx.pairs_of(dx, dy)
        pi.append(i)
        pj.append(j)
        pt.append(np.full(len(i), t, dtype=np.int64))
    if not pi:
        return np.zeros((0, 2), dtype=np.int64), np.zeros(0, dtype=np.int64)
    return np.stack([np.concatenate(pi), np.concatenate(pj)], axis=1), np.concatenate(pt)


def nullity(pos: np.ndarray, types: Sequence[Tuple[int, int]]) -> Tuple[int, int]:
    """Null-space dimensions of the linearised redcal systems (eq. logcal).

    Real parts (amplitudes): ln|V_ij| = eta_i + eta_j + A_alpha.
    Imaginary parts (phases): arg V_ij = phi_i - phi_j + psi_alpha.
    Returns (amplitude nullity, phase nullity); Sec. 5.2 requires 1 + 3.
    """
    pairs, tix = group_pairs(pos, types)
    nant, nt = len(pos), len(types)
    rows = np.arange(len(pairs))
    amp = np.zeros((len(pairs), nant + nt))
    phs = np.zeros((len(pairs), nant + nt))
    amp[rows, pairs[:, 0]] += 1.0
    amp[rows, pairs[:, 1]] += 1.0
    amp[rows, nant + tix] += 1.0
    phs[rows, pairs[:, 0]] += 1.0
    phs[rows, pairs[:, 1]] -= 1.0
    phs[rows, nant + tix] += 1.0
    # rank of the (dense) normal matrices: eigenvalues of A^T A
    na = nant + nt - np.linalg.matrix_rank(amp.T @ amp, hermitian=True)
    nph = nant + nt - np.linalg.matrix_rank(phs.T @ phs, hermitian=True)
    return int(na), int(nph)


def subset_budget(nant: int, p: float = 1.0, log_base: float = math.e) -> float:
    """Pairs a p N log N calibrator can correlate (Sec. 5.5, eq. subredcal_frac_bls)."""
    return p * nant * math.log(nant) / math.log(log_base)


def select_subset(pos: np.ndarray, metric: np.ndarray = SQUARE_METRIC, p: float = 1.0,
                  log_base: float = math.e):
    """Subset redundant-calibration selection (Sec. 5.1 and Sec. 6.1).

    Whole redundant groups are taken in ascending baseline length; the
    prefix whose pair count is closest to p N log N wins (ties go to the
    shorter prefix), and it is extended until the null space holds only the
    four degeneracies of Sec. 5.2.  Returns the list of selected types.
    """
    types, groups = baseline_types(pos, metric)
    budget = subset_budget(len(pos), p, log_base)
    cum = np.cumsum([len(g) for g in groups])
    best = int(np.argmin(np.abs(cum - budget)))     # argmin takes the first (shorter) on ties
    k = best + 1
    while k <= len(types) and sum(nullity(pos, types[:k])) != 4:
        k += 1
    return types[:k]
