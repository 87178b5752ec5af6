"""Predicted statistics of reduced redundant calibration, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2 (gain uncertainty): the linearised (logarithmic) form of eq. redcal
is A x + n = b, and the covariance of the estimate is (A^H N^-1 A)^-1
(eq. cov).  With the same SNR on every visibility, N = SNR^-2 I
(eq. noisecov), and the gain variance is SNR^-2 times the diagonal of the
gains' block of (A^H A)^-1 (eq. gaincov, eq. gaincov_v1).

Reading used here (the paper writes A as one complex matrix and inverts
it, but A^H A is singular along the four degeneracies of Sec. 5.2):

* The logarithm splits the system into two real ones with the same
  sparsity: amplitudes, ln|V_b| = eta_i + eta_j + ln|V_alpha|, and phases,
  arg V_b = phi_i - phi_j + arg V_alpha, for b = (i, j) of type alpha.
* A complex noise n_b with E|n_b|^2 = |V_b|^2 / SNR^2 perturbs ln V_b by
  n_b / V_b, whose real and imaginary parts each have variance
  SNR^-2 / 2.
* The degeneracies are removed the way the gains are compared with the
  truth: mean eta matched (amplitude) and a plane c + k.r fitted to phi and
  removed (phase).  Every solution of the normal equations differs from the
  pseudo-inverse one by a null-space vector, whose gain part lies in
  span{1} (amplitude) or span{1, x, y} (phase); projecting the gains'
  block of the pseudo-inverse off those spans therefore gives the
  covariance of the fixed gains whatever generalised inverse is taken.
* The relative gain error is dg/g = d eta + i d phi, so the predicted
  E|dg/g|^2 per antenna is the sum of the two projected diagonals.

When the amplitude and phase covariances agree this is SNR^-2 times one
of them, eq. gaincov as printed.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def logcal_matrices(pairs: np.ndarray, tix: np.ndarray, n_ant: int, n_types: int) -> Tuple[np.ndarray, np.ndarray]:
    """Real design matrices [N_obs, N + K] of the amplitude and phase halves
    of eq. logcal: columns are the N antennas, then the K types."""
    m = len(pairs)
    rows = np.arange(m)
    a_amp = np.zeros((m, n_ant + n_types))
    a_ph = np.zeros((m, n_ant + n_types))
    a_amp[rows, pairs[:, 0]] += 1.0
    a_amp[rows, pairs[:, 1]] += 1.0
    a_ph[rows, pairs[:, 0]] += 1.0
    a_ph[rows, pairs[:, 1]] -= 1.0
    a_amp[rows, n_ant + tix] = 1.0
    a_ph[rows, n_ant + tix] = 1.0
    return a_amp, a_ph


def _projector_off(basis: np.ndarray) -> np.ndarray:
    """I - Q Q^T for an orthonormal basis Q of span(basis columns)."""
    q, _ = np.linalg.qr(basis)
    return np.eye(basis.shape[0]) - q @ q.T


def gain_covariances(pos: np.ndarray, pairs: np.ndarray, tix: np.ndarray, n_types: int) -> Tuple[np.ndarray, np.ndarray]:
    """(C_eta, C_phi): N x N covariances of the degeneracy-fixed log-amplitude
    and phase errors per unit noise variance of each real equation (eq. cov
    with N = I, gains' block, projected as described above)."""
    n = len(pos)
    a_amp, a_ph = logcal_matrices(pairs, tix, n, n_types)
    r = np.asarray(pos, dtype=float)
    p_amp = _projector_off(np.ones((n, 1)))
    p_ph = _projector_off(np.stack([np.ones(n), r[:, 0], r[:, 1]], axis=1))
    c_amp = np.linalg.pinv(a_amp.T @ a_amp)[:n, :n]
    c_ph = np.linalg.pinv(a_ph.T @ a_ph)[:n, :n]
    return p_amp @ c_amp @ p_amp, p_ph @ c_ph @ p_ph


def predicted_gain_variance(pos: np.ndarray, pairs: np.ndarray, tix: np.ndarray, n_types: int,
                            snr: float) -> np.ndarray:
    """Predicted E|g_est / g_true - 1|^2 per antenna (eq. gaincov, read as
    above): (SNR^-2 / 2) (diag C_eta + diag C_phi)."""
    c_eta, c_phi = gain_covariances(pos, pairs, tix, n_types)
    return (0.5 / snr ** 2) * (np.diag(c_eta) + np.diag(c_phi))


def equations_per_antenna(pairs: np.ndarray, n_ant: int) -> np.ndarray:
    """Number of selected visibilities each antenna takes part in: the
    diagonal of the gains' block of A^T A (Sec. 2, below eq. gaincov)."""
    return np.bincount(pairs.ravel(), minlength=n_ant)


def reduced_chisq(chisq: float, sigma2: float, n_obs: int, n_ant: int, n_ubl: int) -> float:
    """chi^2_r of eq. redchi with one noise variance for every visibility:
    chi^2 / (sigma^2 DoF), DoF = N_obs - N - N_ubl + 2 (eq. dof)."""
    return chisq / (sigma2 * (n_obs - n_ant - n_ubl + 2))



def whole_array_chisq(vfull: np.ndarray, g: np.ndarray, vunique: np.ndarray, pos: np.ndarray, lags) -> Tuple[float, float]:
    """Goodness of fit of the FFT-correlator's model to the full visibility
    matrix (Sec. 2 on the scatter of redundant visibilities, the metric of
    Sec. 6.4): the numerator of eq. redchi over every pair of the array,
    with the gains of the reduced calibration and V^unique (eq. modelvis) as
    the model visibilities.

    vfull: [N, N] visibility matrix of an FX correlator (V_ij, i and j in
    `pos` order); g: [N] gains; vunique: [len(lags)] one value per lag.
    Returns (sum |V_ij - g_i conj(g_j) V_d|^2, sum |V_ij / (g_i conj(g_j)) -
    V_d|^2) over every pair (i, j) with r_i - r_j = d in `lags`.  The second
    (calibrated residuals) has the same sample noise on every pair when the
    voltages are Gaussian, so chi^2_r follows with one sigma^2."""
    from .geometry import PositionIndex
    g = np.asarray(g, dtype=np.complex128)
    idx = PositionIndex(pos)
    c2 = c2cal = 0.0
    for t, (dx, dy) in enumerate(lags):
        i, j = idx.pairs_of(dx, dy)
        gg = g[i] * np.conj(g[j])
        r = vfull[i, j] - gg * vunique[t]
        c2 += float(np.sum(np.abs(r) ** 2))
        c2cal += float(np.sum(np.abs(r / gg) ** 2))
    return c2, c2cal
