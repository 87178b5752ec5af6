"""Statistical validation of the GPU solve at the visibility level (the
simulation of Sec. 3): over many realisations of the true visibilities and
the noise, the spread of the solved gains about the truth must follow the
predicted covariance (eq. gaincov; the oracle's prediction is pinned against
brute force on the CPU), and the reduced chi^2 (eq. redchi, eq. dof) must
be one.  One unit per realisation, all solved in one launch."""
import numpy as np
import pytest
import torch

from oracle import geometry as OG
from oracle import stats as OS
from synthdata.visibilities import simulate_reduced_visibilities

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")


@pytest.mark.parametrize("n,seed", [(8, 21), (16, 22)])
def test_gain_spread_matches_predicted_covariance(rrc, n, seed):
    U, snr = 2048, 100.0
    types, _ = rrc.select_subset(n)
    pos = OG.square_positions(n)
    pairs, tix = OG.group_pairs(pos, types)
    N, K, P = len(pos), len(types), len(pairs)
    vred, g, vm = simulate_reduced_visibilities(seed, pairs, tix, N, K, U, snr)
    plan = rrc.Plan(n, types, U, 256, init_mode="gains", degen_mode="match")
    assert plan.n_pairs == P
    g32 = torch.from_numpy(np.broadcast_to(g.astype(np.complex64), (U, N)).copy()).to(DEV)
    vd = torch.from_numpy(vred.astype(np.complex64)).to(DEV)
    out = plan.solve(vd, gains_in=g32, gains_ref=g32)
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    gg = out["gains"].cpu().numpy().astype(np.complex128)
    gref = g.astype(np.complex64).astype(np.complex128)
    emp = np.mean(np.abs(gg / gref - 1.0) ** 2, axis=0)
    pred = OS.predicted_gain_variance(pos, pairs, tix, K, snr)
    ratio = emp / pred
    chir = OS.reduced_chisq(out["chisq"].cpu().numpy().astype(np.float64), 1.0 / snr ** 2, P, N, K)
    dof = P - N - K + 2
    print(f"n={n}: gain variance / predicted mean {ratio.mean():.4f}, range [{ratio.min():.3f}, "
          f"{ratio.max():.3f}]; chi^2_r mean {chir.mean():.4f}")
    # |dg/g|^2 has two real degrees of freedom: the relative spread of a
    # U-sample mean is 1/sqrt(U) = 2.2% per antenna
    assert abs(ratio.mean() - 1.0) <= 0.03
    assert np.all(np.abs(ratio - 1.0) <= 0.12)
    # chi^2 has 2 DoF real degrees of freedom: spread sqrt(1 / DoF) per unit
    assert abs(chir.mean() - 1.0) <= 4.0 / np.sqrt(U * dof)


def test_gain_variance_falls_with_subset_size(rrc):
    # Fig. 5 (Sec. 5.3): more redundant groups in the subset, lower gain
    # variance.  For each prefix of the length-sorted types, the GPU solve
    # over 1024 realisations against the predicted covariance of that
    # selection (eq. gaincov, the library's rrc_gain_variance, which is
    # pinned to the oracle on the CPU), and the trend itself
    n, U, snr = 8, 1024, 100.0
    allt = OG.square_types(n)[0]
    pos = OG.square_positions(n)
    N = len(pos)
    means = []
    for k, K in enumerate((5, 7, 9, 12, 16)):
        types = [tuple(t) for t in allt[:K]]
        assert sum(OG.nullity(pos, types)) == 4
        pairs, tix = OG.group_pairs(pos, types)
        vred, g, vm = simulate_reduced_visibilities(40 + k, pairs, tix, N, K, U, snr)
        plan = rrc.Plan(n, types, U, 256, init_mode="gains", degen_mode="match")
        g32 = torch.from_numpy(np.broadcast_to(g.astype(np.complex64), (U, N)).copy()).to(DEV)
        out = plan.solve(torch.from_numpy(vred.astype(np.complex64)).to(DEV), gains_in=g32, gains_ref=g32)
        torch.cuda.synchronize()
        assert int((out["status"] != 0).sum()) == 0
        gg = out["gains"].cpu().numpy().astype(np.complex128)
        emp = np.mean(np.abs(gg / g.astype(np.complex64).astype(np.complex128) - 1.0) ** 2, axis=0)
        pred = rrc.gain_variance(n, types, snr)
        ratio = emp.mean() / pred.mean()
        print(f"K={K} ({len(pairs)} pairs): mean gain variance {emp.mean():.3e}, predicted {pred.mean():.3e}, "
              f"ratio {ratio:.4f}")
        assert abs(ratio - 1.0) <= 0.03
        means.append(emp.mean())
    assert all(b < a for a, b in zip(means, means[1:]))


@pytest.mark.parametrize("n,U,T", [(4, 2, 256), (8, 2, 512), (12, 1, 300)])
def test_chisq_full_matches_oracle(rrc, n, U, T):
    # the whole-array fit (Sec. 6.4 metric) on identical complex64 inputs:
    # the oracle's V^full (FX correlator, FP64, all-type pair list), gains
    # and V^unique (eq. modelvis with those gains), each rounded once
    from oracle import correlator as OC
    from tests.gpu_util import make_units
    pos = OG.square_positions(n)
    lags = OC.canonical_lags(n)
    pairs, _ = OG.group_pairs(pos, lags)
    v, g = make_units(n, U, T)
    vf32 = np.empty((U, len(pairs)), dtype=np.complex64)
    vu32 = np.empty((U, len(lags)), dtype=np.complex64)
    g32 = (g * np.exp(0.02j)).astype(np.complex64)
    want = []
    for u in range(U):
        vf = OC.fx_correlate(v[u].astype(np.complex128))
        vf32[u] = vf[pairs[:, 0], pairs[:, 1]].astype(np.complex64)
        vu32[u] = OC.redundant_average(vf, g32[u].astype(np.complex128), pos, lags).astype(np.complex64)
        vfr = np.zeros_like(vf)
        vfr[pairs[:, 0], pairs[:, 1]] = vf32[u].astype(np.complex128)
        want.append(OS.whole_array_chisq(vfr, g32[u].astype(np.complex128), vu32[u].astype(np.complex128), pos, lags))
    c, cc = rrc.chisq_full(n, torch.from_numpy(vf32).to(DEV), torch.from_numpy(g32).to(DEV),
                           torch.from_numpy(vu32).to(DEV))
    c, cc = c.cpu().numpy(), cc.cpu().numpy()
    for u in range(U):
        print(f"n={n} unit {u}: chi2 {c[u]:.6e} (oracle {want[u][0]:.6e}), calibrated {cc[u]:.6e}")
        assert abs(c[u] - want[u][0]) <= 1e-10 * want[u][0]
        assert abs(cc[u] - want[u][1]) <= 1e-10 * want[u][1]


def test_whole_array_chisq_r_near_one(rrc):
    # Sec. 6.4: the reduced calibration's gains with the FFT-correlator's
    # V^unique fit the full visibility matrix with chi^2_r close to one.
    # All on the GPU: the whole path (X-engine, solve, FFT-correlator with
    # the solved gains), V^full from the all-type X-engine over the whole
    # interval, the calibrated residuals summed in FP64.  For Gaussian
    # voltages a calibrated visibility's sample noise is P_i P_j / T
    # (Isserlis), P the calibrated power: V_auto^2 / T for every pair, and
    # independent from pair to pair when the receiver noise dominates the
    # sky (SNR 0.5 per sample; where the sky dominates, pairs sharing
    # antennas carry correlated sample noise and the scatter is smaller).
    # DoF = N_obs - N - N_ubl + 2 (eq. dof) over all N(N-1)/2 pairs.
    from tests.gpu_util import make_units
    n, U, T, snr = 8, 64, 2048, 0.5
    N, K = n * n, 2 * n * (n - 1)
    types, _ = rrc.select_subset(n)
    v, g = make_units(n, U, T, snr=snr)
    vd = torch.from_numpy(v).to(DEV)
    gt = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    plan = rrc.Plan(n, types, U, T)
    out = plan.run(vd, mode="selfcal")
    truth = plan.fftcorr(vd, gt)
    vfull = rrc.LowCadence(n, U, T, one_cycle=True).xengine(vd)
    _, cc = rrc.chisq_full(n, vfull, out["gains"], out["vunique"])
    _, ct = rrc.chisq_full(n, vfull, gt, truth[0])
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    n_obs = N * (N - 1) // 2
    dof = n_obs - N - K + 2
    chir = cc.cpu().numpy() / (out["vauto"].double().cpu().numpy() ** 2 / T * dof)
    chit = ct.cpu().numpy() / (truth[1].double().cpu().numpy() ** 2 / T * dof)
    print(f"chi^2_r against V^full: reduced calibration {chir.mean():.4f} (sd {chir.std():.4f}); "
          f"true gains {chit.mean():.4f}; the groups' scatter alone {(n_obs - K) / dof:.4f}")
    # true gains: only the groups' scatter about their means remains,
    # (N_obs - N_ubl) / DoF on average; |r|^2 / sigma^2 has unit spread per
    # pair, so the mean over U units is within 3 / sqrt(U (N_obs - N_ubl))
    # up to the per-antenna spread of the calibrated power (0.5%)
    assert abs(chit.mean() * dof / (n_obs - K) - 1.0) <= 0.005 + 3.0 / np.sqrt(U * (n_obs - K))
    # the solved gains were fitted to a subset of the same visibilities, so
    # they absorb part of its noise (chi^2 falls below the true gains'), and
    # the fit to the whole array stays close to one
    assert chir.mean() <= chit.mean()
    assert abs(chir.mean() - 1.0) <= 0.05


@pytest.mark.parametrize("side,seed", [(4, 31), (6, 32)])
def test_hex_gain_spread_matches_predicted_covariance(rrc, side, seed):
    # Sec. 3 simulations on the paper's own layout, a hexagonal array: the
    # spread of the masked Gauss-Newton solve's gains over 2048 realisations
    # against eq. gaincov for the hexagon's antennas and pairs
    U, snr = 2048, 100.0
    n, mask = rrc.hex_mask(side)
    _, _, pos = OG.hex_grid(side)
    idx = pos[:, 1] * n + pos[:, 0]
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    pairs, tix = OG.group_pairs(pos, types)
    N, K = len(pos), len(types)
    vred, g, _ = simulate_reduced_visibilities(seed, pairs, tix, N, K, U, snr)
    plan = rrc.Plan(n, types, U, 256, mask=mask, init_mode="gains", degen_mode="match")
    gfull = np.ones(n * n, dtype=np.complex128)
    gfull[idx] = g
    g32 = torch.from_numpy(np.broadcast_to(gfull.astype(np.complex64), (U, n * n)).copy()).to(DEV)
    out = plan.solve(torch.from_numpy(vred.astype(np.complex64)).to(DEV), gains_in=g32, gains_ref=g32)
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    gg = out["gains"].cpu().numpy()[:, idx].astype(np.complex128)
    emp = np.mean(np.abs(gg / g.astype(np.complex64).astype(np.complex128) - 1.0) ** 2, axis=0)
    pred = OS.predicted_gain_variance(pos, pairs, tix, K, snr)
    ratio = emp / pred
    chir = OS.reduced_chisq(out["chisq"].cpu().numpy().astype(np.float64), 1.0 / snr ** 2, len(pairs), N, K)
    dof = len(pairs) - N - K + 2
    print(f"hex side {side} ({N} antennas): gain variance / predicted mean {ratio.mean():.4f}, range "
          f"[{ratio.min():.3f}, {ratio.max():.3f}]; chi^2_r mean {chir.mean():.4f}")
    assert abs(ratio.mean() - 1.0) <= 0.03
    assert np.all(np.abs(ratio - 1.0) <= 0.12)
    assert abs(chir.mean() - 1.0) <= 4.0 / np.sqrt(U * dof)
