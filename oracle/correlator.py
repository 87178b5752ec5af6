"""Direct (FX) correlator, redundant averaging and the reduced X-engine.

TEST INFRASTRUCTURE ONLY (see the package docstring).

All float work is complex128; the 4-bit path is exact int64.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

from .geometry import PositionIndex


def fx_correlate(v: np.ndarray) -> np.ndarray:
    """Full visibility matrix of a traditional FX correlator (Sec. 1).

    v: [T, N] voltages.  Returns V[i, j] = (1/T) sum_t v_i(t) conj(v_j(t)),
    the time-integrated cross-correlation of every antenna pair (the mean
    over the integration; autocorrelations on the diagonal).
    """
    v = np.asarray(v, dtype=np.complex128)
    return (v.T @ v.conj()) / v.shape[0]


def redundant_average(vfull: np.ndarray, gains: np.ndarray, pos: np.ndarray,
                      types: Sequence[Tuple[int, int]]) -> np.ndarray:
    """Calibrated, redundantly averaged visibilities (eq. modelvis).

    V_alpha = (1/N_alpha) sum_{(i,j) in alpha} V_ij / (g_i conj(g_j)),
    with the pairs of type alpha being those with r_i - r_j = d_alpha.
    This is what the FFT-correlator outputs when the voltages are divided
    by the gains before the spatial transform (Sec. 2, Fig. 1).
    A lag that no pair of antennas realises (possible on a masked lattice,
    e.g. a hexagonal array inside its bounding grid) has no visibility; it
    is reported as zero.
    """
    g = np.asarray(gains, dtype=np.complex128)
    idx = PositionIndex(pos)
    out = np.zeros(len(types), dtype=np.complex128)
    for t, (dx, dy) in enumerate(types):
        i, j = idx.pairs_of(dx, dy)
        if len(i):
            out[t] = np.sum(vfull[i, j] / (g[i] * np.conj(g[j]))) / len(i)
    return out


def calibrated_auto(vfull: np.ndarray, gains: np.ndarray) -> float:
    """Zero-lag output: mean over antennas of V_ii / |g_i|^2."""
    g = np.asarray(gains, dtype=np.complex128)
    return float(np.mean(np.real(np.diag(vfull)) / np.abs(g) ** 2))


def xengine(vfull: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Reduced X-engine (Fig. 1 calibrator box): V_ij for the selected pairs only."""
    return vfull[pairs[:, 0], pairs[:, 1]]


def xengine_int(re: np.ndarray, im: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Exact integer X-engine on 4-bit voltages q = re + i im, shape [T, N].

    S_ij = sum_t q_i(t) conj(q_j(t)) as raw int64 sums (no 1/T), returned as
    [P, 2] int64 (real, imaginary).  q_i conj(q_j) = (a_i a_j + b_i b_j)
    + i (b_i a_j - a_i b_j) with q = a + i b.
    """
    # antenna-major copies, so that a pair's samples are contiguous rows
    a = np.ascontiguousarray(np.asarray(re, dtype=np.int64).T)
    b = np.ascontiguousarray(np.asarray(im, dtype=np.int64).T)
    out = np.empty((len(pairs), 2), dtype=np.int64)
    # slices of pairs bound the [pairs, T] gathers' memory
    for s in range(0, len(pairs), 1024):
        i, j = pairs[s:s + 1024, 0], pairs[s:s + 1024, 1]
        ai, aj, bi, bj = a[i], a[j], b[i], b[j]
        out[s:s + 1024, 0] = np.einsum("pt,pt->p", ai, aj) + np.einsum("pt,pt->p", bi, bj)
        out[s:s + 1024, 1] = np.einsum("pt,pt->p", bi, aj) - np.einsum("pt,pt->p", ai, bj)
    return out


def canonical_lags(n: int):
    """Every canonical lag d of an n x n grid in the output order of V^unique.

    Order: d_y ascending, then d_x ascending (d_y = 0 starts at d_x = 1).
    There are 2 n (n - 1) of them.
    """
    out = [(dx, 0) for dx in range(1, n)]
    for dy in range(1, n):
        out += [(dx, dy) for dx in range(-(n - 1), n)]
    return out
