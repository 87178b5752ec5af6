"""Full-size parity in the launch configuration the benchmark times (one plan
for every channel of an array, pipelined run), on sampled units that the
oracle computes one by one: the 16x16-grid, 64-channel, 1024-sample workload
(the benchmark's default) and the 64x64-grid, 1024-channel, 4096-sample
4-bit one.

V^reduced is compared bit for bit on sampled pairs (exact integer sums).  For
V^unique the oracle's redundant average is fed the exact integer
correlations of the sampled lags' pairs, so its cost stays that of a few
lags rather than the full 4096 x 4096 correlation matrix."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from synthdata import WORKLOADS, workload_voltages
from synthdata.device import device_voltages
from synthdata.generate import unpack_ci4
from tests.gpu_util import TOL_GAINS, TOL_VUNIQUE, TOL_XENG, oracle_solve, oracle_vunique, rel_l2

pytestmark = pytest.mark.gpu

UNITS = (5, 901)


def test_bench_workload_sampled_units(rrc):
    # the exact bytes the benchmark feeds (host generator), previous-channel
    # gains as the pipelined FFT's input
    w = {x.name: x for x in WORKLOADS}["g16_c64_t1024"]
    n = w.grids[0]
    U, T = w.n_chan, w.n_time
    v, g = workload_voltages(w, 0)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T)
    dev = torch.device("cuda")
    g64 = g.astype(np.complex64)
    out = plan.run(torch.from_numpy(v).to(dev), gains_in=torch.from_numpy(g64).to(dev), mode="pipelined")
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    pairs, _ = OG.group_pairs(OG.square_positions(n), types)
    for u in (0, 17, 42, 63):
        vf = OC.fx_correlate(v[u].astype(np.complex128))
        vr = out["vred"][u].cpu().numpy()
        ref = OC.xengine(vf, pairs)
        scale = np.mean(np.abs(v[u].astype(np.complex128)) ** 2)
        assert np.max(np.abs(vr - ref)) / scale <= TOL_XENG
        vu_ref, va_ref = oracle_vunique(v[u], g64[u].astype(np.complex128), n)
        assert rel_l2(out["vunique"][u].cpu().numpy(), vu_ref) <= TOL_VUNIQUE
        assert abs(float(out["vauto"][u]) - va_ref) <= 1e-5 * va_ref
        sol = oracle_solve(vr.astype(np.complex128), n, types)
        gg = out["gains"][u].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(gg - sol["g"]) / np.abs(sol["g"]))
        print(f"unit {u}: gains {err:.2e}")
        assert err <= TOL_GAINS
# lag indices in V^unique order: (1,0), (2,0), (63,0), (1,1), (-63,41),
# (63,41), (62,63), (63,63) -- short and long, both signs of dx
LAG_IDX = (0, 1, 62, 63 + 64, 63 + 40 * 127, 63 + 40 * 127 + 126, 2 * 64 * 63 - 2, 2 * 64 * 63 - 1)


def test_ci4_full_workload_sampled_units(rrc):
    w = {x.name: x for x in WORKLOADS}["g64_c1024_t4096_ci4"]
    n = w.grids[0]
    N, U, T = n * n, w.n_chan, w.n_time
    dev = torch.device("cuda")
    volt, g = device_voltages(w, 0, dev)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T, dtype="ci4")
    gin = torch.from_numpy(g.astype(np.complex64)).to(dev)
    out = plan.run(volt, gains_in=gin, mode="pipelined")
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0

    pos = OG.square_positions(n)
    idx = OG.PositionIndex(pos)
    pairs, _ = OG.group_pairs(pos, types)
    lags = OC.canonical_lags(n)
    for u in UNITS:
        re, im = unpack_ci4(volt[u].cpu().numpy())
        # V^reduced bit for bit on 4096 sampled pairs: the first and last
        # 256 (edges of the first and last type) and 3584 drawn at random
        vr = out["vred"][u].cpu().numpy().astype(np.int64)
        P = len(pairs)
        pick = np.concatenate([np.arange(256), np.arange(P - 256, P),
                               np.random.default_rng(u).choice(np.arange(256, P - 256), 3584, replace=False)])
        ref = OC.xengine_int(re, im, pairs[pick])
        assert np.array_equal(vr[pick], ref), f"unit {u}: {int(np.sum(vr[pick] != ref))} mismatches"
        # V^unique at the sampled lags and V_auto, from exact correlations
        vfull = np.zeros((N, N), dtype=np.complex128)
        sel = [lags[k] for k in LAG_IDX]
        for dx, dy in sel:
            i, j = idx.pairs_of(dx, dy)
            s = OC.xengine_int(re, im, np.stack([i, j], axis=1))
            vfull[i, j] = (s[:, 0] + 1j * s[:, 1]) / T
        d = np.arange(N)
        s = OC.xengine_int(re, im, np.stack([d, d], axis=1))
        vfull[d, d] = s[:, 0] / T
        g64 = g[u].astype(np.complex64).astype(np.complex128)
        ref = OC.redundant_average(vfull, g64, pos, sel)
        got = out["vunique"][u].cpu().numpy()[list(LAG_IDX)]
        aref = OC.calibrated_auto(vfull, g64)
        assert abs(float(out["vauto"][u]) - aref) <= 1e-5 * aref
        # The FFT path's error is uniform in the un-normalised correlation
        # C(d) = N_d T V(d): about FP32 rounding times sqrt(M^2) = 128 of the
        # zero lag C(0) = N T V_auto.  Per lag, then, |dV(d)| N_d / (N V_auto)
        # <= 1e-5 (6e-8 x 128, with margin); the lags with few pairs are not
        # held to a relative bound they cannot meet.
        nd = np.array([len(idx.pairs_of(dx, dy)[0]) for dx, dy in sel])
        errn = np.abs(got - ref) * nd / (N * aref)
        print(f"unit {u}: V^unique at {len(sel)} lags, |dV| N_d / (N V_auto) max {errn.max():.2e}, "
              f"relative L2 of the short lags {rel_l2(got[:4], ref[:4]):.2e}")
        assert np.all(errn <= 1e-5)
        assert rel_l2(got[:4], ref[:4]) <= TOL_VUNIQUE
    del volt
    torch.cuda.empty_cache()
