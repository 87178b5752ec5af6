"""Full-size parity in the launch configuration the benchmark times (one plan
for every channel of an array, pipelined run), on sampled units that the
oracle computes one by one: the 16x16-grid, 64-channel, 1024-sample workload
(the benchmark's default), the 32x32-grid, 256-channel one, the uneven batch
of four grids (16 to 48, 128 channels each, run together) and the
64x64-grid, 1024-channel, 4096-sample 4-bit one.

Gains: the whole path's (FP32 X-engine, then the solve) against the oracle's
whole FP64 chain, and the solve of the same launch shape fed the oracle's
V^reduced against the oracle's solve of those values.  For the 4-bit
workload V^reduced is compared bit for bit on every pair (exact integer
sums), so the whole path's gains meet the solver bar directly; the oracle's
redundant average is fed the exact integer correlations of sampled lags'
pairs, so its cost stays that of a few lags rather than the full 4096 x 4096
correlation matrix."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from synthdata import WORKLOADS, workload_voltages
from synthdata.device import device_voltages
from synthdata.generate import unpack_ci4
from tests.gpu_util import (TOL_GAINS, TOL_GAINS_E2E, TOL_VUNIQUE, TOL_XENG, as_c64, gain_err, oracle_solve,
                            oracle_vunique, rel_l2)

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")
WL = {x.name: x for x in WORKLOADS}


def _check_float_unit(out, u, v_unit, g_in, n, types, pairs):
    """V^reduced, V^unique, V_auto and the end-to-end gains of one unit
    against the oracle's own chain; returns the oracle's V^reduced."""
    vf = OC.fx_correlate(v_unit.astype(np.complex128))
    vref = OC.xengine(vf, pairs)
    vr = out["vred"][u].cpu().numpy()
    scale = np.mean(np.abs(v_unit.astype(np.complex128)) ** 2)
    xerr = np.max(np.abs(vr - vref)) / scale
    assert xerr <= TOL_XENG
    vu_ref, va_ref = oracle_vunique(v_unit, g_in.astype(np.complex128), n)
    err_u = rel_l2(out["vunique"][u].cpu().numpy(), vu_ref)
    assert err_u <= TOL_VUNIQUE
    assert abs(float(out["vauto"][u]) - va_ref) <= 1e-5 * va_ref
    sol = oracle_solve(vref, n, types)
    e2e = gain_err(out["gains"][u].cpu().numpy(), sol["g"])
    print(f"n={n} unit {u}: X-engine {xerr:.2e}, V^unique {err_u:.2e}, end-to-end gains {e2e:.2e}")
    assert e2e <= TOL_GAINS_E2E
    return vref


def _check_solver_at_launch_shape(plan, out, units, vrefs, n, types):
    """The plan's solve (the launch rrc_run makes) on its own V^reduced with
    the sampled units' rows replaced by the oracle's, rounded to complex64:
    gains within TOL_GAINS of the oracle's solve of the same values."""
    vr = out["vred"].clone()
    v64 = {}
    for u, x in zip(units, vrefs):
        x32, v64[u] = as_c64(x)
        vr[u] = torch.from_numpy(x32).to(vr.device)
    sol = plan.solve(vr)
    torch.cuda.synchronize()
    for u in units:
        ref = oracle_solve(v64[u], n, types)
        err = gain_err(sol["gains"][u].cpu().numpy(), ref["g"])
        print(f"n={n} unit {u}: solver gains {err:.2e} (niter {int(sol['niter'][u])})")
        assert int(sol["status"][u]) == 0
        assert err <= TOL_GAINS


def test_bench_workload_sampled_units(rrc):
    # the exact bytes the benchmark feeds (host generator)
    w = WL["g16_c64_t1024"]
    n = w.grids[0]
    v, g = workload_voltages(w, 0)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, w.n_chan, w.n_time)
    g32 = g.astype(np.complex64)
    out = plan.run(torch.from_numpy(v).to(DEV), gains_in=torch.from_numpy(g32).to(DEV), mode="pipelined")
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    pairs, _ = OG.group_pairs(OG.square_positions(n), types)
    units = (0, 17, 42, 63)
    vrefs = [_check_float_unit(out, u, v[u], g32[u], n, types, pairs) for u in units]
    _check_solver_at_launch_shape(plan, out, units, vrefs, n, types)


def test_32x32_workload_sampled_units(rrc):
    w = WL["g32_c256_t2048"]
    n = w.grids[0]
    volt, g = device_voltages(w, 0, DEV)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, w.n_chan, w.n_time)
    g32 = g.astype(np.complex64)
    out = plan.run(volt, gains_in=torch.from_numpy(g32).to(DEV), mode="pipelined")
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    pairs, _ = OG.group_pairs(OG.square_positions(n), types)
    units = (3, 200)
    vrefs = [_check_float_unit(out, u, volt[u].cpu().numpy(), g32[u], n, types, pairs) for u in units]
    _check_solver_at_launch_shape(plan, out, units, vrefs, n, types)
    del volt
    torch.cuda.empty_cache()


def test_uneven_batch_workload_sampled_units(rrc):
    w = WL["g16-24-32-48_c128_t1024"]
    plans, volts, gins, outs, gs, tys = [], [], [], [], [], []
    for ai, n in enumerate(w.grids):
        volt, g = device_voltages(w, ai, DEV)
        types, _ = rrc.select_subset(n)
        p = rrc.Plan(n, types, w.n_chan, w.n_time)
        plans.append(p)
        volts.append(volt)
        gs.append(g.astype(np.complex64))
        gins.append(torch.from_numpy(gs[-1]).to(DEV))
        outs.append(p.alloc_outputs(DEV))
        tys.append(types)
    rrc.Batch(plans).run(volts, gins, outs, mode="pipelined")
    torch.cuda.synchronize()
    for ai, n in enumerate(w.grids):
        assert int((outs[ai]["status"] != 0).sum()) == 0
        pairs, _ = OG.group_pairs(OG.square_positions(n), tys[ai])
        units = (7 + 31 * ai, 100 + ai) if n == 48 else (7 + 31 * ai,)
        vrefs = [_check_float_unit(outs[ai], u, volts[ai][u].cpu().numpy(), gs[ai][u], n, tys[ai], pairs)
                 for u in units]
        _check_solver_at_launch_shape(plans[ai], outs[ai], units, vrefs, n, tys[ai])
    del volts
    torch.cuda.empty_cache()


UNITS = (5, 901)
# lag indices in V^unique order: (1,0), (2,0), (63,0), (1,1), (-63,41),
# (63,41), (62,63), (63,63) -- short and long, both signs of dx
LAG_IDX = (0, 1, 62, 63 + 64, 63 + 40 * 127, 63 + 40 * 127 + 126, 2 * 64 * 63 - 2, 2 * 64 * 63 - 1)


def test_ci4_full_workload_sampled_units(rrc):
    w = WL["g64_c1024_t4096_ci4"]
    n = w.grids[0]
    N, U, T = n * n, w.n_chan, w.n_time
    volt, g = device_voltages(w, 0, DEV)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T, dtype="ci4")
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    out = plan.run(volt, gains_in=gin, mode="pipelined")
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0

    pos = OG.square_positions(n)
    idx = OG.PositionIndex(pos)
    pairs, _ = OG.group_pairs(pos, types)
    lags = OC.canonical_lags(n)
    for u in UNITS:
        re, im = unpack_ci4(volt[u].cpu().numpy())
        # V^reduced bit for bit on every pair; the gains against the oracle's
        # solve of the same exact integer sums (the whole path's input to
        # the solve is then identical on both sides)
        vr = out["vred"][u].cpu().numpy().astype(np.int64)
        ref = OC.xengine_int(re, im, pairs)
        assert np.array_equal(vr, ref), f"unit {u}: {int(np.sum(vr != ref))} mismatches"
        sol = oracle_solve(ref[:, 0] + 1j * ref[:, 1], n, types)
        gerr = gain_err(out["gains"][u].cpu().numpy(), sol["g"])
        print(f"unit {u}: gains {gerr:.2e} (niter {int(out['niter'][u])})")
        assert gerr <= TOL_GAINS
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
