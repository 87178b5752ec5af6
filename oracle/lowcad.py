"""Low-cadence calibration (Sec. 4), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The calibrator correlates about p N log N baselines at a time (the
O(N log N) budget of eq. lowcadcal_inttime) and cycles through all of them:
after N_cycle cycles the full visibility matrix is populated and redundant
calibration runs on it once.  Each cycle integrates t_int = t_cal / N_cycle
of the calibration interval, and every pair of one redundant group is
correlated in the same cycle, so redundancy is preserved (Sec. 4).

Readings (the paper gives neither the order of the round robin nor how a
cycle is filled):
* groups are taken in the lag order of V^unique (dy ascending, then dx;
  dy = 0 starts at dx = 1), and a cycle takes whole groups in that order
  while its pair count stays within p N ln N (a group larger than the
  budget would take a cycle alone; none is on a square grid of N >= 4);
* cycle c integrates samples [floor(c T / N_cycle), floor((c+1) T / N_cycle))
  of the interval's T samples, and its visibilities are the mean over them;
* calibration of the populated matrix is the same redundant calibration as
  for a reduced set (redcal.calibrate), over every type.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from . import geometry as G
from .correlator import canonical_lags


def budget(n_ant: int, p: float = 1.0, log_base: float = math.e) -> float:
    """Pairs correlated per cycle: p N log N (eq. lowcadcal_inttime)."""
    return p * n_ant * math.log(n_ant) / math.log(log_base)


def schedule(n: int, p: float = 1.0, log_base: float = math.e) -> List[Tuple[int, int]]:
    """Cycles as ranges [t0, t1) of lag-order types, whole groups per cycle."""
    lags = canonical_lags(n)
    b = budget(n * n, p, log_base)
    cycles, start, cnt = [], 0, 0
    for t, (dx, dy) in enumerate(lags):
        m = (n - abs(dx)) * (n - dy)
        if cnt > 0 and cnt + m > b:
            cycles.append((start, t))
            start, cnt = t, 0
        cnt += m
    cycles.append((start, len(lags)))
    return cycles


def sample_ranges(n_time: int, n_cycles: int) -> List[Tuple[int, int]]:
    """Samples [s0, s1) integrated by each cycle (t_int = T / N_cycle)."""
    return [(c * n_time // n_cycles, (c + 1) * n_time // n_cycles) for c in range(n_cycles)]


def visibilities(v: np.ndarray, n: int, cycles) -> np.ndarray:
    """The populated visibility matrix as the all-type pair list.

    v: [T, N] voltages of one integration interval.  Pairs are type-major in
    lag order, within a type by the raster index of the first antenna
    (group_pairs); pair (i, j) of cycle c is (1/t_c) sum over the cycle's
    samples of v_i conj(v_j), the FX correlator over those samples.
    """
    v = np.asarray(v, dtype=np.complex128)
    lags = canonical_lags(n)
    pos = G.square_positions(n)
    pairs, tix = G.group_pairs(pos, lags)
    out = np.empty(len(pairs), dtype=np.complex128)
    for (t0, t1), (s0, s1) in zip(cycles, sample_ranges(v.shape[0], len(cycles))):
        sel = (tix >= t0) & (tix < t1)
        i, j = pairs[sel, 0], pairs[sel, 1]
        out[sel] = np.einsum("tp,tp->p", v[s0:s1, i], np.conj(v[s0:s1, j])) / (s1 - s0)
    return out
