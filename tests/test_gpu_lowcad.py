"""Low-cadence calibration on the GPU (Sec. 4) against the oracle: the
round-robin X-engine populating every pair from its cycle's samples, and the
omnical solve over every type reaching the oracle's Gauss-Newton minimum."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import lowcad as OL
from tests.gpu_util import TOL_OMNICAL, TOL_XENG, as_c64, gain_err, make_units, oracle_solve

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")


@pytest.mark.parametrize("n,U,T,p", [(4, 2, 300, 1.0), (8, 1, 512, 1.0), (8, 2, 97, 0.5), (16, 1, 1024, 1.0)])
def test_lowcad_xengine_matches_oracle(rrc, n, U, T, p):
    v, _ = make_units(n, U, T, wid=120 + n)
    lc = rrc.LowCadence(n, U, T, p=p)
    assert lc.cycles == OL.schedule(n, p)
    got = lc.xengine(torch.from_numpy(v).to(DEV)).cpu().numpy()
    for u in range(U):
        ref = OL.visibilities(v[u].astype(np.complex128), n, lc.cycles)
        scale = np.mean(np.abs(v[u].astype(np.complex128)) ** 2)
        err = np.max(np.abs(got[u] - ref)) / scale
        print(f"n={n} p={p} unit {u}: {len(lc.cycles)} cycles, max err / power {err:.2e}")
        assert err <= TOL_XENG


@pytest.mark.parametrize("n,U,T", [(6, 2, 512), (8, 2, 1024)])
def test_lowcad_solve_matches_oracle(rrc, n, U, T):
    v, g = make_units(n, U, T, wid=130 + n)
    lc = rrc.LowCadence(n, U, T)
    lags = OC.canonical_lags(n)
    vr32 = np.empty((U, lc.n_pairs), np.complex64)
    vr64 = []
    for u in range(U):
        vr32[u], x = as_c64(OL.visibilities(v[u].astype(np.complex128), n, lc.cycles))
        vr64.append(x)
    out = lc.solve(torch.from_numpy(vr32).to(DEV), torch.from_numpy(g.astype(np.complex64)).to(DEV))
    torch.cuda.synchronize()
    for u in range(U):
        ref = oracle_solve(vr64[u], n, lags)
        gerr = gain_err(out["gains"][u].cpu().numpy(), ref["g"])
        cerr = abs(float(out["chisq"][u]) - ref["chisq"]) / ref["chisq"]
        print(f"n={n} unit {u}: gains {gerr:.2e} chi2 {cerr:.2e} niter {int(out['niter'][u])} "
              f"status {int(out['status'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_OMNICAL
        assert cerr <= 1e-5
