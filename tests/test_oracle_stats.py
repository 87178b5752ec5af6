"""Pins of the oracle's predicted calibration statistics (Sec. 2, gain
uncertainty; eq. cov, eq. noisecov, eq. gaincov, eq. gainvar_redcal,
eq. redchi, eq. dof) against brute force and the paper's closed forms."""
import numpy as np
import pytest

from oracle import geometry as OG
from oracle import redcal as OR
from oracle import stats as OS
from synthdata.visibilities import simulate_reduced_visibilities


def _full(n):
    pos = OG.square_positions(n)
    types, _ = OG.square_types(n)
    pairs, tix = OG.group_pairs(pos, types)
    return pos, types, pairs, tix


def test_equations_per_antenna_full_matrix_is_n_minus_one():
    # with every pair, each antenna takes part in N - 1 visibilities (the
    # diagonal the paper quotes as ~N below eq. gaincov); brute-force count
    pos, types, pairs, tix = _full(5)
    n = len(pos)
    a_amp, a_ph = OS.logcal_matrices(pairs, tix, n, len(types))
    count = np.array([sum(1 for i, j in pairs if k in (i, j)) for k in range(n)])
    assert np.array_equal(OS.equations_per_antenna(pairs, n), count)
    assert np.all(count == n - 1)
    assert np.array_equal(np.diag(a_amp.T @ a_amp)[:n], count)
    assert np.array_equal(np.diag(a_ph.T @ a_ph)[:n], count)


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_full_matrix_gain_variance_follows_one_over_n(n):
    # eq. gainvar_redcal: with the full visibility matrix sigma_g^2 ~ SNR^-2 / N;
    # the finite-N excess shrinks like 1/N
    pos, types, pairs, tix = _full(n)
    N = len(pos)
    v = OS.predicted_gain_variance(pos, pairs, tix, len(types), snr=1.0)
    assert abs(N * v.mean() - 1.0) <= 2.0 / N
    # and SNR enters as SNR^-2
    assert np.allclose(OS.predicted_gain_variance(pos, pairs, tix, len(types), snr=10.0), v / 100.0)


def test_null_space_has_the_four_degeneracies():
    # the projected covariances are finite only because A^T A's null space is
    # exactly the degeneracies of Sec. 5.2: one amplitude, three phase
    pos = OG.square_positions(5)
    types = OG.select_subset_square(5)
    pairs, tix = OG.group_pairs(pos, types)
    a_amp, a_ph = OS.logcal_matrices(pairs, tix, len(pos), len(types))
    k = len(pos) + len(types)
    assert k - np.linalg.matrix_rank(a_amp) == 1
    assert k - np.linalg.matrix_rank(a_ph) == 3
    assert OG.nullity(pos, types) == (1, 3)


def test_predicted_variance_matches_monte_carlo_of_the_nonlinear_solve():
    # brute force: the oracle's Gauss-Newton solve (not linearised) over many
    # noise and sky realisations, degeneracies matched to the true gains as in
    # Sec. 3, against the prediction; also chi^2_r -> 1 (eq. redchi, eq. dof)
    n, snr, R = 5, 100.0, 300
    pos = OG.square_positions(n)
    types = OG.select_subset_square(n)
    pairs, tix = OG.group_pairs(pos, types)
    N, K = len(pos), len(types)
    vred, g, vm = simulate_reduced_visibilities(11, pairs, tix, N, K, R, snr)
    err2 = np.zeros(N)
    chir = []
    for r in range(R):
        sol = OR.calibrate(vred[r], pos, types, pairs, tix, init=(g, vm[r]), fix="match", g_ref=g)
        assert sol["converged"]
        err2 += np.abs(sol["g"] / g - 1.0) ** 2
        chir.append(OS.reduced_chisq(sol["chisq"], 1.0 / snr ** 2, len(pairs), N, K))
    emp = err2 / R
    pred = OS.predicted_gain_variance(pos, pairs, tix, K, snr)
    ratio = emp / pred
    # |dg/g|^2 has two real degrees of freedom: the relative spread of an
    # R-sample mean is 1/sqrt(R) = 5.8% per antenna
    assert abs(ratio.mean() - 1.0) <= 0.05, ratio.mean()
    assert np.all(np.abs(ratio - 1.0) <= 0.25), ratio
    # chi^2 has 2 DoF real degrees of freedom: spread sqrt(1 / DoF) per draw
    assert abs(np.mean(chir) - 1.0) <= 4.0 / np.sqrt(R * OR.dof(len(pairs), N, K))


def test_fixed_gain_errors_carry_no_degenerate_component():
    # after the degeneracy fix of Sec. 3 the log-amplitude errors have zero
    # mean and the phase errors no plane c + k.r, in every draw; the sample
    # covariances of the brute-force solve annihilate those directions, and
    # so must the predicted ones
    n, snr, R = 5, 100.0, 40
    pos = OG.square_positions(n)
    types = OG.select_subset_square(n)
    pairs, tix = OG.group_pairs(pos, types)
    N, K = len(pos), len(types)
    vred, g, vm = simulate_reduced_visibilities(12, pairs, tix, N, K, R, snr)
    eta, phi = [], []
    for r in range(R):
        sol = OR.calibrate(vred[r], pos, types, pairs, tix, init=(g, vm[r]), fix="match", g_ref=g)
        q = sol["g"] / g
        eta.append(np.log(np.abs(q)))
        phi.append(np.angle(q))
    eta, phi = np.array(eta), np.array(phi)
    r = np.asarray(pos, dtype=float)
    plane = np.stack([np.ones(N), r[:, 0], r[:, 1]], axis=1)
    c_eta, c_phi = OS.gain_covariances(pos, pairs, tix, K)
    scale_e, scale_p = np.abs(eta).max() ** 2, np.abs(phi).max() ** 2
    assert np.abs(eta.T @ eta @ np.ones(N)).max() <= 1e-9 * R * N * scale_e
    assert np.abs(phi.T @ phi @ plane).max() <= 1e-9 * R * N * scale_p * np.abs(plane).max()
    assert np.abs(c_eta @ np.ones(N)).max() <= 1e-10 * np.abs(c_eta).max()
    assert np.abs(c_phi @ plane).max() <= 1e-10 * np.abs(c_phi).max() * np.abs(plane).max()


def test_subset_raises_the_predicted_variance():
    # Sec. 5: calibrating on a subset of the baseline types (a sub-matrix of A)
    # gives a larger gain variance than the full matrix, and more types help
    n = 8
    pos = OG.square_positions(n)
    full_types, _ = OG.square_types(n)
    vs = []
    for k in (4, 6, 10, len(full_types)):
        types = full_types[:k]
        if OG.nullity(pos, types) != (1, 3):
            continue
        pairs, tix = OG.group_pairs(pos, types)
        vs.append(OS.predicted_gain_variance(pos, pairs, tix, k, 1.0).mean())
    assert len(vs) >= 3
    assert all(a > b for a, b in zip(vs, vs[1:]))


def test_whole_array_chisq_pins():
    # (1) noise-free redundant data is fitted exactly; (2) with V_d the group
    # mean of the calibrated visibilities, the calibrated sum is the groups'
    # scatter about their means (N_d times the population variance); (3) any
    # other model value raises it (the group mean is the least-squares fit)
    from oracle import correlator as C
    from oracle import stats as S
    n = 4
    pos = OG.square_positions(n)
    lags = C.canonical_lags(n)
    rng = np.random.default_rng(8)
    g = (1 + 0.1 * rng.standard_normal(n * n)) * np.exp(1j * rng.uniform(-3, 3, n * n))
    vd = rng.standard_normal(len(lags)) + 1j * rng.standard_normal(len(lags))
    vf = np.zeros((n * n, n * n), dtype=np.complex128)
    idx = OG.PositionIndex(pos)
    for t, d in enumerate(lags):
        i, j = idx.pairs_of(*d)
        vf[i, j] = g[i] * np.conj(g[j]) * vd[t]
    c2, c2cal = S.whole_array_chisq(vf, g, vd, pos, lags)
    assert c2 < 1e-24 and c2cal < 1e-24
    noisy = vf + 0.1 * (rng.standard_normal(vf.shape) + 1j * rng.standard_normal(vf.shape))
    vmean = C.redundant_average(noisy, g, pos, lags)
    _, c2cal = S.whole_array_chisq(noisy, g, vmean, pos, lags)
    scatter = 0.0
    for t, d in enumerate(lags):
        i, j = idx.pairs_of(*d)
        q = noisy[i, j] / (g[i] * np.conj(g[j]))
        scatter += len(q) * (np.var(q.real) + np.var(q.imag))
    assert abs(c2cal - scatter) <= 1e-10 * scatter
    for _ in range(5):
        bump = vmean + 0.01 * (rng.standard_normal(len(lags)) + 1j * rng.standard_normal(len(lags)))
        assert S.whole_array_chisq(noisy, g, bump, pos, lags)[1] > c2cal
