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
