"""Masked lattices on the GPU: hexagonal arrays (Sec. 3, Fig. 2) laid on
their lattice index grid, against the FP64 oracle fed the same antennas.

The voltages are the seeded sky on the whole grid; only the hexagon's grid
points are antennas, and the oracle sees exactly those (in raster order,
its positions `oracle.geometry.hex_grid`).  V^unique keeps every lag of the
grid (zero where no pair realises it); V^reduced and the solve cover the
mask's pairs only."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import redcal as OR
from tests.gpu_util import TOL_OMNICAL, TOL_VUNIQUE, TOL_XENG, as_c64, gain_err, make_ci4_units, make_units, rel_l2

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _hex(rrc, side):
    n, mask = rrc.hex_mask(side)
    n2, m2, pos = OG.hex_grid(side)
    assert n == n2 and np.array_equal(mask.astype(bool), m2)
    return n, mask, pos, pos[:, 1] * n + pos[:, 0]


def _embedded(side, n):
    # the hexagon in the lower-left corner of a larger n x n grid (4-bit
    # plans need n*n a multiple of 4 and an even n)
    _, _, hp = OG.hex_grid(side)
    mask = np.zeros(n * n, dtype=np.uint8)
    mask[hp[:, 1] * n + hp[:, 0]] = 1
    return mask, hp, hp[:, 1] * n + hp[:, 0]


@pytest.mark.parametrize("side,U,T", [(2, 2, 64), (3, 2, 200), (4, 2, 256), (6, 1, 333), (11, 2, 512),
                                      (17, 1, 64), (4, 1, 1), (20, 2, 100), (24, 1, 1)])
def test_hex_fftcorr_matches_oracle(rrc, side, U, T):
    n, mask, pos, idx = _hex(rrc, side)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    plan = rrc.Plan(n, types, U, T, mask=mask)
    assert plan.info["masked"] == 1 and plan.info["n_live"] == len(pos)
    v, g = make_units(n, U, T)
    g64 = g.astype(np.complex64)
    vu, va = plan.fftcorr(torch.from_numpy(v).to(DEV), torch.from_numpy(g64).to(DEV))
    vu, va = vu.cpu().numpy(), va.cpu().numpy()
    lags = OC.canonical_lags(n)
    for u in range(U):
        vf = OC.fx_correlate(v[u][:, idx].astype(np.complex128))
        gl = g64[u][idx].astype(np.complex128)
        ref = OC.redundant_average(vf, gl, pos, lags)
        aref = OC.calibrated_auto(vf, gl)
        empty = np.array([len(OG.PositionIndex(pos).pairs_of(dx, dy)[0]) == 0 for dx, dy in lags])
        err = rel_l2(vu[u], ref)
        print(f"hex side {side} (n={n}, N={len(pos)}) T={T} unit {u}: V^unique rel L2 {err:.2e}, "
              f"{int(empty.sum())} empty lags")
        assert err <= TOL_VUNIQUE
        assert np.all(vu[u][empty] == 0)
        assert abs(va[u] - aref) <= 1e-5 * aref


@pytest.mark.parametrize("side,U,T,m", [(11, 2, 256, 64), (9, 1, 100, 64), (12, 1, 64, 64), (20, 1, 64, 128),
                                        (24, 2, 33, 128)])
def test_hex_fftcorr_power_of_two_size_matches_oracle(rrc, side, U, T, m):
    # the default is the mixed-radix size (48 up to 12 antennas a side, 96 up
    # to 24); the power of two beside it
    n, mask, pos, idx = _hex(rrc, side)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    plan = rrc.Plan(n, types, U, T, mask=mask)
    assert plan.info["fft_size"] == m * 3 // 4
    plan.set_fft_size(m)
    v, g = make_units(n, U, T)
    g64 = g.astype(np.complex64)
    vu, va = plan.fftcorr(torch.from_numpy(v).to(DEV), torch.from_numpy(g64).to(DEV))
    vu, va = vu.cpu().numpy(), va.cpu().numpy()
    lags = OC.canonical_lags(n)
    empty = np.array([len(OG.PositionIndex(pos).pairs_of(dx, dy)[0]) == 0 for dx, dy in lags])
    for u in range(U):
        vf = OC.fx_correlate(v[u][:, idx].astype(np.complex128))
        gl = g64[u][idx].astype(np.complex128)
        ref = OC.redundant_average(vf, gl, pos, lags)
        err = rel_l2(vu[u], ref)
        print(f"M={m} hex side {side} (n={n}) T={T} unit {u}: V^unique rel L2 {err:.2e}")
        assert err <= TOL_VUNIQUE
        assert np.all(vu[u][empty] == 0)
        assert abs(va[u] - OC.calibrated_auto(vf, gl)) <= 1e-5 * OC.calibrated_auto(vf, gl)


@pytest.mark.parametrize("side,U,T", [(3, 2, 300), (4, 2, 1024), (11, 1, 512)])
def test_hex_xengine_float_matches_oracle(rrc, side, U, T):
    n, mask, pos, idx = _hex(rrc, side)
    types, npairs = rrc.select_subset_masked(n, mask, "hex")
    pairs, tix = OG.group_pairs(pos, types)
    assert len(pairs) == npairs
    plan = rrc.Plan(n, types, U, T, mask=mask)
    assert plan.n_pairs == npairs
    v, _ = make_units(n, U, T)
    vr = plan.xengine(torch.from_numpy(v).to(DEV)).cpu().numpy()
    for u in range(U):
        ref = OC.xengine(OC.fx_correlate(v[u][:, idx].astype(np.complex128)), pairs)
        scale = np.mean(np.abs(v[u][:, idx]) ** 2)
        err = float(np.max(np.abs(vr[u] - ref)) / scale)
        print(f"hex side {side} unit {u}: V^reduced max |dV| / <|v|^2> {err:.2e} ({npairs} pairs)")
        assert err <= TOL_XENG


@pytest.mark.parametrize("side,n,U,T", [(4, 8, 2, 256), (6, 12, 1, 130), (11, 24, 1, 64)])
def test_hex_xengine_ci4_bit_exact(rrc, side, n, U, T):
    mask, pos, idx = _embedded(side, n)
    types, npairs = rrc.select_subset_masked(n, mask, "hex")
    pairs, _ = OG.group_pairs(pos, types)
    plan = rrc.Plan(n, types, U, T, dtype="ci4", mask=mask)
    b, re, im, _ = make_ci4_units(n, U, T)
    vr = plan.xengine(torch.from_numpy(b).to(DEV)).cpu().numpy()
    for u in range(U):
        ref = OC.xengine_int(re[u][:, idx].astype(np.int64), im[u][:, idx].astype(np.int64), pairs)
        assert np.array_equal(vr[u].astype(np.int64), ref), f"unit {u}"
    print(f"hex side {side} on {n}x{n}: {npairs} pairs bit-exact")


@pytest.mark.parametrize("side,n", [(4, 8), (11, 24), (17, 34), (17, 36)])
def test_hex_fftcorr_ci4_matches_oracle(rrc, side, n):
    U, T = 1, 128
    mask, pos, idx = _embedded(side, n)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    plan = rrc.Plan(n, types, U, T, dtype="ci4", mask=mask)
    b, re, im, g = make_ci4_units(n, U, T)
    g64 = g.astype(np.complex64)
    vu, va = plan.fftcorr(torch.from_numpy(b).to(DEV), torch.from_numpy(g64).to(DEV))
    v = re[0][:, idx].astype(np.complex128) + 1j * im[0][:, idx].astype(np.complex128)
    vf = OC.fx_correlate(v)
    gl = g64[0][idx].astype(np.complex128)
    ref = OC.redundant_average(vf, gl, pos, OC.canonical_lags(n))
    err = rel_l2(vu.cpu().numpy()[0], ref)
    print(f"ci4 hex side {side} on {n}x{n}: V^unique rel L2 {err:.2e}")
    assert err <= TOL_VUNIQUE
    assert abs(float(va[0]) - OC.calibrated_auto(vf, gl)) <= 1e-5 * OC.calibrated_auto(vf, gl)


@pytest.mark.parametrize("side,U,T", [(3, 2, 512), (4, 2, 1024), (6, 1, 1024)])
def test_hex_omnical_reaches_the_oracle_minimum(rrc, side, U, T):
    # the masked omnical (from the true gains) and the oracle's Gauss-Newton
    # (FP64, from the same start) reach the same minimum of eq. redchi, with
    # the degeneracies fixed against the first antenna in raster order and
    # its +x, +y neighbours on both sides
    n, mask, pos, idx = _hex(rrc, side)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    pairs, tix = OG.group_pairs(pos, types)
    plan = rrc.Plan(n, types, U, T, mask=mask)
    v, g = make_units(n, U, T, snr=10.0)
    vr32 = np.empty((U, len(pairs)), dtype=np.complex64)
    vr64 = np.empty((U, len(pairs)), dtype=np.complex128)
    for u in range(U):
        vr32[u], vr64[u] = as_c64(OC.xengine(OC.fx_correlate(v[u][:, idx].astype(np.complex128)), pairs))
    st = plan.omnical(torch.from_numpy(vr32).to(DEV), gains_in=torch.from_numpy(g.astype(np.complex64)).to(DEV),
                      max_iter=20000, tol=1e-7)
    torch.cuda.synchronize()
    gg = st["gains"].cpu().numpy()
    dead = np.ones(n * n, dtype=bool)
    dead[idx] = False
    for u in range(U):
        gl = g[u][idx]
        ref = OR.calibrate(vr64[u], pos, types, pairs, tix, init=(gl, OR.group_mean(vr64[u], gl, pairs, tix, len(types))))
        gerr = gain_err(gg[u][idx], ref["g"])
        cerr = abs(float(st["chisq"][u]) - ref["chisq"]) / ref["chisq"]
        print(f"hex side {side} unit {u}: omnical gains {gerr:.2e} chi2 {cerr:.2e} niter {int(st['niter'][u])}")
        assert int(st["status"][u]) == 0
        assert gerr <= TOL_OMNICAL
        assert cerr <= 1e-5
        assert np.all(gg[u][dead] == 0)


def test_masked_full_grid_equals_plain_plan(rrc):
    # a mask with every grid point set is the square grid: the same
    # V^unique, V^reduced and omnical result as the plain plan
    n, U, T = 8, 2, 256
    types, _ = rrc.select_subset(n)
    v, g = make_units(n, U, T)
    vd, gd = torch.from_numpy(v).to(DEV), torch.from_numpy(g.astype(np.complex64)).to(DEV)
    a = rrc.Plan(n, types, U, T)
    b = rrc.Plan(n, types, U, T, mask=np.ones(n * n, dtype=np.uint8))
    assert a.n_pairs == b.n_pairs
    for x, y in zip(a.fftcorr(vd, gd), b.fftcorr(vd, gd)):
        assert torch.equal(x, y)
    va, vb = a.xengine(vd), b.xengine(vd)
    assert torch.equal(va, vb)
    sa = a.omnical(va, gains_in=gd, max_iter=300, tol=0.0)
    sb = b.omnical(vb, gains_in=gd, max_iter=300, tol=0.0)
    for k in ("gains", "vmodel", "chisq", "niter"):
        assert torch.equal(sa[k], sb[k]), k


def _hex_solve_case(rrc, side, U, T, snr=10.0, **opts):
    n, mask, pos, idx = _hex(rrc, side)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    pairs, tix = OG.group_pairs(pos, types)
    plan = rrc.Plan(n, types, U, T, mask=mask, init_mode="gains", **opts)
    v, g = make_units(n, U, T, snr=snr)
    vr32 = np.empty((U, len(pairs)), dtype=np.complex64)
    vr64 = np.empty((U, len(pairs)), dtype=np.complex128)
    for u in range(U):
        vr32[u], vr64[u] = as_c64(OC.xengine(OC.fx_correlate(v[u][:, idx].astype(np.complex128)), pairs))
    return n, mask, pos, idx, types, pairs, tix, plan, v, g, vr32, vr64


@pytest.mark.parametrize("side,U,T", [(3, 2, 512), (4, 2, 1024), (6, 2, 1024), (11, 1, 2048), (14, 1, 1024)])
def test_hex_gauss_newton_matches_oracle(rrc, side, U, T):
    # the adjoint-driven Gauss-Newton solve on a masked lattice, started from
    # the true gains, against the oracle's FP64 solve of the same (rounded)
    # V^reduced, both fixed against the first antenna and its neighbours
    from tests.gpu_util import TOL_GAINS
    n, mask, pos, idx, types, pairs, tix, plan, v, g, vr32, vr64 = _hex_solve_case(rrc, side, U, T)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    out = plan.solve(torch.from_numpy(vr32).to(DEV), gains_in=gin)
    torch.cuda.synchronize()
    gg = out["gains"].cpu().numpy()
    dead = np.ones(n * n, dtype=bool)
    dead[idx] = False
    for u in range(U):
        gl = g[u][idx]
        ref = OR.calibrate(vr64[u], pos, types, pairs, tix,
                           init=(gl, OR.group_mean(vr64[u], gl, pairs, tix, len(types))))
        gerr = gain_err(gg[u][idx], ref["g"])
        cerr = abs(float(out["chisq"][u]) - ref["chisq"]) / ref["chisq"]
        print(f"hex side {side} unit {u}: Gauss-Newton gains {gerr:.2e} chi2 {cerr:.2e} "
              f"steps {int(out['niter'][u])} dof {plan.dof} (oracle {ref['dof']})")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS
        assert cerr <= 1e-5
        assert plan.dof == ref["dof"]
        assert np.all(gg[u][dead] == 0)


def test_hex_gauss_newton_match_mode(rrc):
    # MATCH: the mean log-amplitude and the phase plane of the reference
    # gains (the paper's procedure), on the hexagon's antennas only
    from tests.gpu_util import TOL_GAINS
    side, U, T = 4, 2, 1024
    n, mask, pos, idx, types, pairs, tix, plan, v, g, vr32, vr64 = _hex_solve_case(rrc, side, U, T,
                                                                                     degen_mode="match")
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    out = plan.solve(torch.from_numpy(vr32).to(DEV), gains_in=gin, gains_ref=gin)
    torch.cuda.synchronize()
    for u in range(U):
        gl = g[u].astype(np.complex64).astype(np.complex128)[idx]
        ref = OR.calibrate(vr64[u], pos, types, pairs, tix, fix="match", g_ref=gl,
                           init=(gl, OR.group_mean(vr64[u], gl, pairs, tix, len(types))))
        gerr = gain_err(out["gains"][u].cpu().numpy()[idx], ref["g"])
        print(f"hex side {side} unit {u}: MATCH gains {gerr:.2e}")
        assert gerr <= TOL_GAINS


@pytest.mark.parametrize("mode", ["selfcal", "pipelined"])
def test_hex_whole_path_run(rrc, mode):
    # rrc_run on a hexagonal array: X-engine, Gauss-Newton from the given
    # gains, FFT-correlator; against the oracle's whole FP64 chain
    from tests.gpu_util import TOL_GAINS_E2E
    side, U, T = 6, 2, 1024
    n, mask, pos, idx, types, pairs, tix, plan, v, g, vr32, vr64 = _hex_solve_case(rrc, side, U, T)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    out = plan.run(torch.from_numpy(v).to(DEV), gains_in=gin, mode=mode)
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    lags = OC.canonical_lags(n)
    for u in range(U):
        vf = OC.fx_correlate(v[u][:, idx].astype(np.complex128))
        assert np.max(np.abs(out["vred"][u].cpu().numpy() - OC.xengine(vf, pairs))) <= TOL_XENG * np.mean(
            np.abs(v[u][:, idx]) ** 2)
        gl = g[u][idx]
        vr = OC.xengine(vf, pairs)
        ref = OR.calibrate(vr, pos, types, pairs, tix, init=(gl, OR.group_mean(vr, gl, pairs, tix, len(types))))
        gerr = gain_err(out["gains"][u].cpu().numpy()[idx], ref["g"])
        # the FFT-correlator applied the solved gains (selfcal) or the given ones (pipelined)
        gfft = ref["g"] if mode == "selfcal" else g[u].astype(np.complex64).astype(np.complex128)[idx]
        vref = OC.redundant_average(vf, gfft, pos, lags)
        verr = rel_l2(out["vunique"][u].cpu().numpy(), vref)
        print(f"{mode} hex side {side} unit {u}: gains {gerr:.2e}, V^unique {verr:.2e}")
        assert gerr <= TOL_GAINS_E2E
        assert verr <= TOL_VUNIQUE


def test_masked_full_grid_solve_equals_plain_plan(rrc):
    # a full mask runs the same Gauss-Newton arithmetic as the plain plan
    n, U, T = 8, 2, 256
    types, _ = rrc.select_subset(n)
    v, g = make_units(n, U, T)
    vd, gd = torch.from_numpy(v).to(DEV), torch.from_numpy(g.astype(np.complex64)).to(DEV)
    a = rrc.Plan(n, types, U, T, init_mode="gains")
    b = rrc.Plan(n, types, U, T, mask=np.ones(n * n, dtype=np.uint8), init_mode="gains")
    oa = a.run(vd, gains_in=gd, mode="selfcal")
    ob = b.run(vd, gains_in=gd, mode="selfcal")
    torch.cuda.synchronize()
    for k in ("vred", "gains", "vmodel", "chisq", "niter", "status", "vunique", "vauto"):
        assert torch.equal(oa[k], ob[k]), k


def test_hex_tuner_keeps_results(rrc, tmp_path):
    # the autotuner on the 331-antenna hexagon (21 x 21 grid: the 48-point
    # transform is a candidate); the tuned run's V^reduced and solve are the
    # untuned ones bit for bit, V^unique meets the oracle
    side, U, T = 11, 4, 512
    n, mask, pos, idx = _hex(rrc, side)
    types, _ = rrc.select_subset_masked(n, mask, "hex")
    plan = rrc.Plan(n, types, U, T, mask=mask, init_mode="gains")
    v, g = make_units(n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    ref = plan.run(vd, gains_in=gin, mode="pipelined")
    cache = str(tmp_path / "tune.txt")
    t1 = plan.tune(vd, gin, cache_path=cache)
    assert t1["from_cache"] == 0 and t1["fft_size"] in (48, 64)
    got = plan.run(vd, gains_in=gin, mode="pipelined", out=plan.alloc_outputs(DEV))
    torch.cuda.synchronize()
    for key in ("vred", "gains", "vmodel", "chisq", "niter", "status"):
        assert torch.equal(got[key], ref[key]), key
    lags = OC.canonical_lags(n)
    for u in range(U):
        vf = OC.fx_correlate(v[u][:, idx].astype(np.complex128))
        want = OC.redundant_average(vf, g[u].astype(np.complex64).astype(np.complex128)[idx], pos, lags)
        assert rel_l2(got["vunique"][u].cpu().numpy(), want) <= TOL_VUNIQUE
    # another mask on the same grid shape does not take this choice
    other = mask.copy()
    other[np.flatnonzero(other)[0]] = 0
    types2, _ = rrc.select_subset_masked(n, other, "hex")
    p2 = rrc.Plan(n, types2, U, T, mask=other, init_mode="gains")
    assert p2.tune(vd, gin, cache_path=cache)["from_cache"] == 0
    p3 = rrc.Plan(n, types, U, T, mask=mask, init_mode="gains")
    t3 = p3.tune(vd, gin, cache_path=cache)
    assert t3["from_cache"] == 1 and t3["fft_size"] == t1["fft_size"]
    print(f"hex side {side}: tuned {t1}")
