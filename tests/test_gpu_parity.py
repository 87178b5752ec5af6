"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import redcal as OR
from tests.gpu_util import (TOL_GAINS, TOL_GAINS_E2E, TOL_OMNICAL, TOL_VUNIQUE, TOL_XENG, as_c64, ci4_sums_int32,
                            gain_err,
                            make_ci4_units, make_units, oracle_solve, oracle_vred, oracle_vunique, pairs_of,
                            rel_l2)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _plan(rrc, n, U, T, dtype="c64", types=None, **kw):
    if types is None:
        types, _ = rrc.select_subset(n)
    return rrc.Plan(n, types, U, T, dtype=dtype, **kw), types


# ------------------------------------------------------------------ (a1)-(a3)

@pytest.mark.parametrize("n,U,T", [(8, 1, 256), (16, 6, 1024), (3, 2, 37), (5, 3, 250),
                                   (12, 2, 333), (24, 2, 200), (32, 2, 512), (40, 1, 33),
                                   (48, 2, 64), (64, 1, 40), (16, 1, 4096), (33, 1, 31), (45, 2, 17),
                                   (3, 1, 1), (16, 2, 1), (40, 1, 1)])
def test_fftcorr_matches_oracle(rrc, n, U, T):
    v, g = make_units(n, U, T)
    plan, _ = _plan(rrc, n, U, T)
    g64 = g.astype(np.complex64)
    vu, va = plan.fftcorr(torch.from_numpy(v).to(DEV), torch.from_numpy(g64).to(DEV))
    vu, va = vu.cpu().numpy(), va.cpu().numpy()
    for u in range(U):
        ref, aref = oracle_vunique(v[u], g64[u].astype(np.complex128), n)
        err = rel_l2(vu[u], ref)
        print(f"n={n} T={T} unit {u}: V^unique rel L2 {err:.2e}, auto {abs(va[u] - aref) / aref:.2e}")
        assert err <= TOL_VUNIQUE
        assert abs(va[u] - aref) <= 1e-5 * aref


@pytest.mark.parametrize("n,U,T", [(16, 2, 256), (64, 1, 40), (34, 1, 21), (36, 2, 64), (64, 2, 131)])
def test_fftcorr_ci4_matches_oracle(rrc, n, U, T):
    # 4-bit voltages: the oracle is fed the same integers
    b, re, im, g = make_ci4_units(n, U, T)
    plan, _ = _plan(rrc, n, U, T, dtype="ci4")
    g64 = g.astype(np.complex64)
    vu, va = plan.fftcorr(torch.from_numpy(b).to(DEV), torch.from_numpy(g64).to(DEV))
    vu, va = vu.cpu().numpy(), va.cpu().numpy()
    for u in range(U):
        v = re[u].astype(np.complex128) + 1j * im[u].astype(np.complex128)
        ref, aref = oracle_vunique(v, g64[u].astype(np.complex128), n)
        err = rel_l2(vu[u], ref)
        print(f"ci4 n={n} T={T} unit {u}: V^unique rel L2 {err:.2e}")
        assert err <= TOL_VUNIQUE
        assert abs(va[u] - aref) <= 1e-5 * aref


@pytest.mark.parametrize("n,U,T,dtype", [(17, 2, 131, "c64"), (20, 1, 64, "c64"), (24, 2, 200, "c64"),
                                         (23, 1, 1, "c64"), (20, 2, 77, "ci4"), (24, 1, 256, "ci4"),
                                         (33, 2, 70, "c64"), (40, 1, 129, "c64"), (45, 2, 37, "c64"),
                                         (48, 2, 256, "c64"), (47, 1, 1, "c64"), (34, 1, 22, "ci4"),
                                         (44, 2, 96, "ci4"), (48, 1, 301, "ci4")])
def test_fftcorr_both_sizes_match_oracle(rrc, n, U, T, dtype):
    # 17 <= n <= 24 and 33 <= n <= 48: the mixed-radix default (48 = 3 x 16,
    # 96 = 3 x 32) and the power of two beside it; 2n - 1 <= M keeps the
    # circular correlation free of wrap-around at either size
    if dtype == "ci4":
        b, re, im, g = make_ci4_units(n, U, T)
        vd = torch.from_numpy(b).to(DEV)
        v = re.astype(np.complex128) + 1j * im.astype(np.complex128)
    else:
        v, g = make_units(n, U, T)
        vd = torch.from_numpy(v).to(DEV)
    plan, _ = _plan(rrc, n, U, T, dtype=dtype)
    mixed = 48 if n <= 24 else 96
    assert plan.info["fft_size"] == mixed
    g64 = g.astype(np.complex64)
    refs = [oracle_vunique(v[u], g64[u].astype(np.complex128), n) for u in range(U)]
    for m in (mixed, {48: 64, 96: 128}[mixed]):
        plan.set_fft_size(m)
        assert plan.info["fft_size"] == m
        vu, va = plan.fftcorr(vd, torch.from_numpy(g64).to(DEV))
        vu, va = vu.cpu().numpy(), va.cpu().numpy()
        for u in range(U):
            ref, aref = refs[u]
            err = rel_l2(vu[u], ref)
            print(f"M={m} {dtype} n={n} T={T} unit {u}: V^unique rel L2 {err:.2e}")
            assert err <= TOL_VUNIQUE
            assert abs(va[u] - aref) <= 1e-5 * aref


@pytest.mark.parametrize("n,m,k0", [(24, 48, (5, 29)), (48, 96, (7, 61))])
def test_fftcorr_mixed_radix_single_mode_closed_form(rrc, n, m, k0):
    # a sky mode on the M-point frequency grid, unit gains, no noise:
    # V(d) = <|s|^2> exp(-2 pi i k0.d / M)
    T = 40
    rng = np.random.default_rng(m)
    s = (rng.standard_normal(T) + 1j * rng.standard_normal(T))
    k0 = np.array(k0)
    pos = OG.square_positions(n)
    v = (s[:, None] * np.exp(-2j * np.pi * (pos @ k0) / m)[None, :]).astype(np.complex64)[None]
    plan, _ = _plan(rrc, n, 1, T)
    assert plan.info["fft_size"] == m
    vu, _ = plan.fftcorr(torch.from_numpy(v).to(DEV), torch.ones((1, n * n), dtype=torch.complex64, device=DEV))
    p = np.mean(np.abs(v[0, :, 0].astype(np.complex128)) ** 2)
    ref = np.array([p * np.exp(-2j * np.pi * (k0 @ np.array(d)) / m) for d in OC.canonical_lags(n)])
    assert rel_l2(vu.cpu().numpy()[0], ref) <= TOL_VUNIQUE


def test_fftcorr_single_mode_closed_form(rrc):
    # one sky mode, no noise, unit gains: V(d) = <|s|^2> exp(-2 pi i k0.d / M)
    n, T, m = 16, 64, 32
    rng = np.random.default_rng(5)
    s = (rng.standard_normal(T) + 1j * rng.standard_normal(T))
    k0 = np.array([3, 7])
    pos = OG.square_positions(n)
    v = (s[:, None] * np.exp(-2j * np.pi * (pos @ k0) / m)[None, :]).astype(np.complex64)[None]
    plan, _ = _plan(rrc, n, 1, T)
    vu, _ = plan.fftcorr(torch.from_numpy(v).to(DEV), torch.ones((1, n * n), dtype=torch.complex64, device=DEV))
    p = np.mean(np.abs(v[0, :, 0]) ** 2)
    ref = np.array([p * np.exp(-2j * np.pi * (k0 @ np.array(d)) / m) for d in OC.canonical_lags(n)])
    assert rel_l2(vu.cpu().numpy()[0], ref) <= TOL_VUNIQUE


# ----------------------------------------------------------------------- (a4)

@pytest.mark.parametrize("n,U,T", [(8, 1, 256), (16, 4, 1024), (5, 2, 97), (32, 2, 2048), (3, 2, 1), (16, 1, 1)])
def test_xengine_float_matches_oracle(rrc, n, U, T):
    v, _ = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    vr = plan.xengine(torch.from_numpy(v).to(DEV)).cpu().numpy()
    pairs, _ = pairs_of(n, types)
    for u in range(U):
        ref = OC.xengine(OC.fx_correlate(v[u].astype(np.complex128)), pairs)
        scale = np.mean(np.abs(v[u].astype(np.complex128)) ** 2)
        err = np.max(np.abs(vr[u] - ref)) / scale
        print(f"n={n} T={T} unit {u}: X-engine max err / power {err:.2e}")
        assert err <= TOL_XENG


@pytest.mark.parametrize("kind", ["mfma", "dot"])
@pytest.mark.parametrize("n,U,T", [(8, 2, 300), (8, 3, 301), (12, 2, 130), (16, 1, 1027), (16, 2, 1024),
                                   (24, 2, 96), (32, 1, 200), (48, 1, 64), (64, 2, 4096), (4, 1, 1), (64, 1, 1)])
def test_xengine_ci4_bit_exact(rrc, n, U, T, kind):
    # the int8 matrix-core and the 4-bit dot-product kernels, both exact
    b, re, im, _ = make_ci4_units(n, U, T)
    plan, types = _plan(rrc, n, U, T, dtype="ci4")
    plan.set_xengine(kind)
    vr = plan.xengine(torch.from_numpy(b).to(DEV)).cpu().numpy().astype(np.int64)
    pairs, _ = pairs_of(n, types)
    for u in range(U):
        ref = OC.xengine_int(re[u], im[u], pairs)
        assert np.array_equal(vr[u], ref), f"unit {u}: {np.sum(vr[u] != ref)} mismatches"


@pytest.mark.parametrize("kind", ["mfma", "dot"])
@pytest.mark.parametrize("n,T", [(8, 259), (16, 1024), (64, 300)])
def test_xengine_ci4_full_nibble_range(rrc, n, T, kind):
    # every byte value, so both nibbles take -8 .. 7 (the -8 products included)
    from synthdata.generate import unpack_ci4
    rng = np.random.default_rng(17)
    b = rng.integers(0, 256, size=(2, T, n * n), dtype=np.uint8)
    b[:, :4, :] = 0x88                       # (-8, -8) at the start of each unit
    plan, types = _plan(rrc, n, 2, T, dtype="ci4")
    plan.set_xengine(kind)
    vr = plan.xengine(torch.from_numpy(b).to(DEV)).cpu().numpy().astype(np.int64)
    pairs, _ = pairs_of(n, types)
    for u in range(2):
        re, im = unpack_ci4(b[u])
        ref = OC.xengine_int(re, im, pairs)
        assert np.array_equal(vr[u], ref), f"unit {u}: {np.sum(vr[u] != ref)} mismatches"


# ----------------------------------------------------------------------- (a5)
#
# The solve is fed the oracle's own V^reduced (FP64 X-engine of the FX
# matrix, or exact integer sums for 4-bit data), rounded to complex64 by the
# test; the oracle solves the same rounded values promoted to FP64.

def _solve_case(rrc, n, U, T, snr, wid=90):
    v, _ = make_units(n, U, T, snr=snr, wid=wid)
    plan, types = _plan(rrc, n, U, T)
    pairs, _ = pairs_of(n, types)
    vr32 = np.empty((U, len(pairs)), np.complex64)
    vr64 = []
    for u in range(U):
        vr32[u], x = as_c64(oracle_vred(v[u], pairs))
        vr64.append(x)
    return plan, types, vr32, vr64


@pytest.mark.parametrize("n,U,T,snr", [(8, 1, 256, 10.0), (16, 4, 1024, 10.0), (24, 2, 512, 10.0),
                                       (32, 2, 2048, 5.0), (48, 2, 1024, 10.0)])
def test_solve_matches_oracle(rrc, n, U, T, snr):
    plan, types, vr32, vr64 = _solve_case(rrc, n, U, T, snr)
    out = plan.solve(torch.from_numpy(vr32).to(DEV))
    for u in range(U):
        ref = oracle_solve(vr64[u], n, types)
        gerr = gain_err(out["gains"][u].cpu().numpy(), ref["g"])
        cerr = abs(float(out["chisq"][u]) - ref["chisq"]) / ref["chisq"]
        verr = np.max(np.abs(out["vmodel"][u].cpu().numpy() - ref["vm"]) / np.abs(ref["vm"]))
        print(f"n={n} unit {u}: gains {gerr:.2e} vmodel {verr:.2e} chi2 {cerr:.2e} "
              f"niter {int(out['niter'][u])} status {int(out['status'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS
        assert verr <= 1e-5
        assert cerr <= 1e-5


@pytest.mark.parametrize("n", [24, 48, 64])
def test_solve_large_grid_recovers_noise_free_gains(rrc, n):
    # V_b = g_i conj(g_j) V_alpha (eq. redcal without noise), rounded to
    # complex64: GPU and oracle solve the same rounded values, and both land
    # within rounding of the injected truth, at the sizes of the uneven-batch
    # and 4-bit workloads (several antennas per work-item, up to 9 types)
    U = 2
    types, _ = rrc.select_subset(n)
    pos = OG.square_positions(n)
    pairs, tix = pairs_of(n, types)
    rng = np.random.default_rng(1000 + n)
    vred = np.empty((U, len(pairs)), np.complex64)
    truth, v64 = [], []
    for u in range(U):
        g = (1 + 0.05 * rng.standard_normal(n * n)) * np.exp(1j * rng.uniform(-np.pi, np.pi, n * n))
        vm = (0.2 + rng.random(len(types))) * np.exp(1j * rng.uniform(-np.pi, np.pi, len(types)))
        vred[u], x = as_c64(OR.model_vis(g, vm, pairs, tix))
        v64.append(x)
        truth.append(OR.fix_refant(g, vm, pos, types)[0])
    plan = rrc.Plan(n, types, U, 64)
    out = plan.solve(torch.from_numpy(vred).to(DEV))
    for u in range(U):
        ref = oracle_solve(v64[u], n, types)
        gerr = gain_err(out["gains"][u].cpu().numpy(), ref["g"])
        terr = float(np.max(np.abs(ref["g"] - truth[u]) / np.abs(truth[u])))
        print(f"n={n} unit {u}: gains {gerr:.2e} (oracle vs truth {terr:.2e}) niter {int(out['niter'][u])} "
              f"status {int(out['status'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS
        assert terr <= 1e-5


@pytest.mark.parametrize("n,U,T", [(16, 2, 1024), (64, 2, 4096)])
def test_solve_ci4_matches_oracle(rrc, n, U, T):
    # 4-bit: the solve reads exact int32 sums; the oracle's integer X-engine
    # gives the very same integers
    b, re, im, _ = make_ci4_units(n, U, T)
    plan, types = _plan(rrc, n, U, T, dtype="ci4")
    pairs, _ = pairs_of(n, types)
    sums = [OC.xengine_int(re[u], im[u], pairs) for u in range(U)]
    vr = np.stack([ci4_sums_int32(x) for x in sums])
    out = plan.solve(torch.from_numpy(vr).to(DEV))
    for u in range(U):
        ref = oracle_solve(sums[u][:, 0] + 1j * sums[u][:, 1], n, types)
        gerr = gain_err(out["gains"][u].cpu().numpy(), ref["g"])
        print(f"ci4 n={n} unit {u}: gains {gerr:.2e} niter {int(out['niter'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS


def test_solve_from_gains_and_match_mode(rrc):
    n, U, T = 16, 2, 1024
    v, gtrue = make_units(n, U, T)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T, init_mode="gains", degen_mode="match")
    pairs, tix = pairs_of(n, types)
    vr32 = np.empty((U, len(pairs)), np.complex64)
    vr64 = []
    for u in range(U):
        vr32[u], x = as_c64(oracle_vred(v[u], pairs))
        vr64.append(x)
    gin = torch.from_numpy(gtrue.astype(np.complex64)).to(DEV)
    out = plan.solve(torch.from_numpy(vr32).to(DEV), gains_in=gin, gains_ref=gin)
    for u in range(U):
        gref = gtrue[u].astype(np.complex64).astype(np.complex128)
        # matching phases is only well posed near the reference: start both there
        ref = oracle_solve(vr64[u], n, types, fix="match", g_ref=gref,
                           init=(gref, OR.group_mean(vr64[u], gref, pairs, tix, len(types))))
        assert gain_err(out["gains"][u].cpu().numpy(), ref["g"]) <= TOL_GAINS
        assert int(out["status"][u]) == 0


@pytest.mark.parametrize("n,U,T", [(8, 2, 256), (16, 2, 1024)])
def test_omnical_reaches_the_oracle_minimum(rrc, n, U, T):
    # omnical's damped updates (FP32, from the true gains) and the oracle's
    # Gauss-Newton (FP64, from its FIRSTCAL start) reach the same minimum of
    # eq. redchi; FP32 stops at a relative change of 1e-7, so the gains agree
    # to FP32 rounding times the iteration's condition
    plan, types, vr32, vr64 = _solve_case(rrc, n, U, T, 10.0)
    _, g = make_units(n, U, T, snr=10.0, wid=90)
    st = plan.omnical(torch.from_numpy(vr32).to(DEV), gains_in=torch.from_numpy(g.astype(np.complex64)).to(DEV),
                      max_iter=20000, tol=1e-7)
    torch.cuda.synchronize()
    for u in range(U):
        ref = oracle_solve(vr64[u], n, types)
        gerr = gain_err(st["gains"][u].cpu().numpy(), ref["g"])
        cerr = abs(float(st["chisq"][u]) - ref["chisq"]) / ref["chisq"]
        print(f"n={n} unit {u}: omnical gains {gerr:.2e} chi2 {cerr:.2e} niter {int(st['niter'][u])} "
              f"status {int(st['status'][u])}")
        assert int(st["status"][u]) == 0
        assert gerr <= TOL_OMNICAL
        assert cerr <= 1e-5


def test_omnical_host_stepped_equals_one_call(rrc):
    # the plain form (one iteration per call, state carried) is the same
    # arithmetic as one call of many iterations
    n, U, T = 8, 2, 256
    plan, types, vr32, _ = _solve_case(rrc, n, U, T, 10.0)
    _, g = make_units(n, U, T, snr=10.0, wid=90)
    vr = torch.from_numpy(vr32).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    a = plan.omnical(vr, gains_in=gin, max_iter=7, tol=0.0, finish=True)
    b = plan.omnical(vr, gains_in=gin, max_iter=1, tol=0.0, finish=False)
    for _ in range(5):
        b = plan.omnical(vr, max_iter=1, tol=0.0, finish=False, state=b)
    b = plan.omnical(vr, max_iter=1, tol=0.0, finish=True, state=b)
    torch.cuda.synchronize()
    assert torch.equal(b["niter"], a["niter"]) and int(a["niter"][0]) == 7
    for k in ("gains", "vmodel", "chisq"):
        assert torch.equal(a[k], b[k]), k


def test_solve_nonfinite_unit_is_flagged(rrc):
    n, U, T = 8, 2, 128
    v, _ = make_units(n, U, T)
    v[1, 5, 7] = np.nan
    plan, _ = _plan(rrc, n, U, T)
    out = plan.run(torch.from_numpy(v).to(DEV), mode="selfcal")
    st = out["status"].cpu().numpy()
    assert st[0] == 0 and st[1] == 2


# ----------------------------------------------------------------------- (a6)
#
# Inputs: the oracle's V^reduced rounded to complex64, gains near the truth
# and group means; the oracle evaluates the same rounded values in FP64.
# Sizes cover the three work-item shapes of the kernel (one, four and
# sixteen antennas per work-item: up to 256, 1024 and 4096 antennas).

def _chisq_case(n, U, T, seed, snr=10.0):
    v, gtrue = make_units(n, U, T, snr=snr)
    types = OG.select_subset_square(n)
    pairs, tix = pairs_of(n, types)
    rng = np.random.default_rng(seed)
    vr32 = np.empty((U, len(pairs)), np.complex64)
    g = (gtrue * (1 + 0.03 * (rng.standard_normal(gtrue.shape) + 1j * rng.standard_normal(gtrue.shape)))
         ).astype(np.complex64)
    vm = np.empty((U, len(types)), np.complex64)
    for u in range(U):
        vr32[u], x = as_c64(oracle_vred(v[u], pairs))
        vm[u] = OR.group_mean(x, gtrue[u], pairs, tix, len(types)).astype(np.complex64)
    return types, pairs, tix, vr32, g, vm


@pytest.mark.parametrize("n,U,T", [(16, 3, 512), (32, 2, 256), (64, 1, 64)])
def test_chisq_and_adjoint_match_oracle(rrc, n, U, T):
    types, pairs, tix, vr32, g, vm = _chisq_case(n, U, T, seed=3)
    plan = rrc.Plan(n, types, U, T)
    gd, vmd, vrd = (torch.from_numpy(x).to(DEV) for x in (g, vm, vr32))
    c = plan.chisq_fwd(gd, vmd, vrd).cpu().numpy()
    gg, gv, dg, dv = [x.cpu().numpy() for x in plan.chisq_adj(gd, vmd, vrd)]
    for u in range(U):
        g64, v64, r64 = g[u].astype(np.complex128), vm[u].astype(np.complex128), vr32[u].astype(np.complex128)
        cref = OR.chisq(r64, g64, v64, pairs, tix)
        rg, rv = OR.wirtinger_grad(r64, g64, v64, pairs, tix)
        hg, hv = OR.jhj_diag(g64, v64, pairs, tix)
        errs = (abs(c[u] - cref) / cref, np.max(np.abs(gg[u] - 2 * rg)) / np.max(np.abs(2 * rg)),
                np.max(np.abs(gv[u] - 2 * rv)) / np.max(np.abs(2 * rv)),
                np.max(np.abs(dg[u] - hg) / hg), np.max(np.abs(dv[u] - hv) / hv))
        print(f"n={n} unit {u}: chi2 {errs[0]:.2e} grad_g {errs[1]:.2e} grad_v {errs[2]:.2e} "
              f"diag_g {errs[3]:.2e} diag_v {errs[4]:.2e}")
        assert max(errs) <= 1e-5


@pytest.mark.parametrize("n,T,snr", [(8, 256, 10.0), (32, 2048, 5.0), (64, 64, 10.0)])
def test_adjoint_matches_central_finite_differences(rrc, n, T, snr):
    # chi^2 is quadratic in each single complex parameter (no pair has
    # i = j), so central differences of the FP64 chi^2 with step 1e-3 are
    # exact up to rounding: d chi2/d Re z + i d chi2/d Im z = 2 d chi2/d conj(z),
    # which is what rrc_chisq_adj returns.  32x32 at SNR 5 and 2048 samples
    # is the 256-channel workload's unit.
    types, pairs, tix, vr32, g, vm = _chisq_case(n, 1, T, seed=11, snr=snr)
    plan = rrc.Plan(n, types, 1, T)
    gg, gv, _, _ = plan.chisq_adj(*(torch.from_numpy(x).to(DEV) for x in (g, vm, vr32)))
    gg, gv = gg.cpu().numpy()[0], gv.cpu().numpy()[0]
    g64, v64, vr = g[0].astype(np.complex128), vm[0].astype(np.complex128), vr32[0].astype(np.complex128)
    h = 1e-3

    def fd(which, k):
        out = 0j
        for unit in (1.0, 1j):
            gp, gm, vp, vmn = g64.copy(), g64.copy(), v64.copy(), v64.copy()
            if which == "g":
                gp[k] += h * unit
                gm[k] -= h * unit
            else:
                vp[k] += h * unit
                vmn[k] -= h * unit
            d = (OR.chisq(vr, gp, vp, pairs, tix) - OR.chisq(vr, gm, vmn, pairs, tix)) / (2 * h)
            out += d * unit
        return out

    rng = np.random.default_rng(11)
    sc_g = np.max(np.abs(gg))
    for k in list(rng.choice(n * n, size=8, replace=False)) + [0, n * n - 1]:
        assert abs(gg[k] - fd("g", k)) <= 1e-5 * sc_g, k
    sc_v = np.max(np.abs(gv))
    for k in range(len(types)):
        assert abs(gv[k] - fd("v", k)) <= 1e-5 * sc_v, k


def test_chisq_autograd_function(rrc):
    n, U, T = 8, 2, 256
    types, pairs, tix, vr32, g0, _ = _chisq_case(n, U, T, seed=4)
    plan = rrc.Plan(n, types, U, T)
    vr_d = torch.from_numpy(vr32).to(DEV)
    g = torch.from_numpy(g0).to(DEV).requires_grad_(True)
    vm = torch.full((U, len(types)), 0.3 + 0.1j, dtype=torch.complex64, device=DEV).requires_grad_(True)
    w = torch.tensor([0.7, 1.3], device=DEV)
    loss = (rrc.chisq(g, vm, vr_d, plan) * w).sum()
    loss.backward()
    gg, gv, _, _ = plan.chisq_adj(g.detach(), vm.detach(), vr_d)
    assert torch.allclose(g.grad, gg * w[:, None], rtol=1e-6, atol=0)
    assert torch.allclose(vm.grad, gv * w[:, None], rtol=1e-6, atol=0)


# ---------------------------------------------------------------- whole path

def test_run_modes_consistent(rrc):
    n, U, T = 16, 3, 1024
    v, gtrue = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(gtrue.astype(np.complex64)).to(DEV)
    a = plan.run(vd, gains_in=gin, mode="pipelined")
    vu_a, _ = plan.fftcorr(vd, gin)
    assert torch.equal(a["vunique"], vu_a)
    b = plan.run(vd, mode="selfcal")
    vu_b, _ = plan.fftcorr(vd, b["gains"].contiguous())
    assert torch.equal(b["vunique"], vu_b)
    assert torch.equal(a["gains"], b["gains"])
    # end to end against the oracle's own chain: its FP64 X-engine, its
    # solve, and its redundant average with its own gains (eq. modelvis)
    pairs, _ = pairs_of(n, types)
    for u in range(U):
        ref = oracle_solve(oracle_vred(v[u], pairs), n, types)
        gerr = gain_err(b["gains"][u].cpu().numpy(), ref["g"])
        vref, _ = oracle_vunique(v[u], ref["g"], n)
        verr = rel_l2(b["vunique"][u].cpu().numpy(), vref)
        print(f"unit {u}: end-to-end gains {gerr:.2e}, V^unique {verr:.2e}")
        assert gerr <= TOL_GAINS_E2E
        assert verr <= TOL_VUNIQUE


@pytest.mark.parametrize("dtype", ["c64", "ci4"])
def test_run_matches_separate_stages_bitwise(rrc, dtype):
    # the whole path in one call gives the same bits as the stages called
    # one at a time (X-engine with several time chunks, solve from its output)
    n, U, T = 16, 3, 1024
    if dtype == "ci4":
        b, _, _, _ = make_ci4_units(n, U, T)
        vd = torch.from_numpy(b).to(DEV)
    else:
        v, _ = make_units(n, U, T)
        vd = torch.from_numpy(v).to(DEV)
    plan, _ = _plan(rrc, n, U, T, dtype=dtype)
    a = plan.run(vd, mode="selfcal")
    vr = plan.xengine(vd)
    assert torch.equal(a["vred"], vr)
    s = plan.solve(vr)
    for k in ("gains", "vmodel", "chisq", "niter", "status"):
        assert torch.equal(a[k], s[k]), k


def test_repeat_is_bitwise_deterministic(rrc):
    n, U, T = 16, 4, 512
    v, _ = make_units(n, U, T)
    plan, _ = _plan(rrc, n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    a = plan.run(vd, mode="selfcal")
    b = plan.run(vd, mode="selfcal", out=plan.alloc_outputs(DEV))
    for k in ("vunique", "vred", "gains", "vmodel", "chisq"):
        assert torch.equal(a[k], b[k]), k


def test_lanes_on_separate_streams_match_serial_runs(rrc):
    # several batches in flight: one plan, stream, input and output set per
    # lane, steps launched round-robin with no synchronisation between them,
    # give the bits of each batch run alone
    n, U, T, D = 16, 8, 512, 3
    lanes = []
    for k in range(D):
        v, g = make_units(n, U, T, wid=300 + k)
        p, _ = _plan(rrc, n, U, T)
        lanes.append(dict(plan=p, v=torch.from_numpy(v).to(DEV), g=torch.from_numpy(g.astype(np.complex64)).to(DEV),
                          out=p.alloc_outputs(DEV), stream=torch.cuda.Stream(DEV)))
    ref = []
    for ln in lanes:
        p1, _ = _plan(rrc, n, U, T)
        ref.append(p1.run(ln["v"], gains_in=ln["g"], mode="pipelined"))
    torch.cuda.synchronize()
    start = torch.cuda.Event()
    start.record()
    for ln in lanes:
        ln["stream"].wait_event(start)
    for i in range(3 * D):
        ln = lanes[i % D]
        with torch.cuda.stream(ln["stream"]):
            ln["plan"].run(ln["v"], gains_in=ln["g"], mode="pipelined", out=ln["out"])
    torch.cuda.synchronize()
    for ln, r in zip(lanes, ref):
        for k in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "niter", "status"):
            assert torch.equal(ln["out"][k], r[k]), k


# ------------------------------------------------------------ uneven batches

def _batch_inputs(rrc):
    shapes = [(8, 3, 256), (12, 2, 300), (16, 4, 512), (5, 2, 97)]
    plans, volts, gins = [], [], []
    for k, (n, U, T) in enumerate(shapes):
        v, g = make_units(n, U, T, wid=200 + k)
        p, _ = _plan(rrc, n, U, T)
        plans.append(p)
        volts.append(torch.from_numpy(v).to(DEV))
        gins.append(torch.from_numpy(g.astype(np.complex64)).to(DEV))
    return plans, volts, gins


def test_batch_matches_eager_runs(rrc):
    # arrays of different grids (and chunkings) run concurrently on branch
    # streams; every repeat, with eager work and synchronisation in between,
    # must equal the plans run one by one (all kernels are deterministic)
    plans, volts, gins = _batch_inputs(rrc)
    for mode in ("pipelined", "selfcal"):
        ref = [p.run(v, gains_in=gi, mode=mode) for p, v, gi in zip(plans, volts, gins)]
        torch.cuda.synchronize()
        batch = rrc.Batch(plans)
        outs = [p.alloc_outputs(DEV) for p in plans]
        for rep in range(3):
            for o in outs:
                for t in o.values():
                    t.fill_(7)                      # eager work between repeats
            batch.run(volts, gins, outs, mode=mode)
            torch.cuda.synchronize()
            for k, (o, r) in enumerate(zip(outs, ref)):
                for key in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "status"):
                    assert torch.equal(o[key], r[key]), (mode, rep, k, key)
        del batch


@pytest.mark.skip(reason="RRC_BATCH_GRAPH is switched off (rrc_batch_create returns RRC_ENOTIMPL): "
                         "capturing the batch's fork/join over its branch and auxiliary streams into a HIP "
                         "graph ended the test process with a host segmentation fault inside rrc_batch_run, "
                         "also after the graph-instantiate out-parameters were given storage; no cause in "
                         "this library has been shown")
def test_batch_graph_matches_eager_runs(rrc):
    # the whole uneven batch captured once (fork/join over branch and
    # auxiliary streams) and replayed as one graph launch: every replay, with
    # eager work and synchronisation in between, equals the eager runs
    plans, volts, gins = _batch_inputs(rrc)
    ref = [p.run(v, gains_in=gi, mode="pipelined") for p, v, gi in zip(plans, volts, gins)]
    torch.cuda.synchronize()
    batch = rrc.Batch(plans, graph=True)
    outs = [p.alloc_outputs(DEV) for p in plans]
    for rep in range(4):
        for o in outs:
            for t in o.values():
                t.fill_(7)
        torch.cuda.synchronize()
        batch.run(volts, gins, outs, mode="pipelined")
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, ref)):
            for key in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "niter", "status"):
                assert torch.equal(o[key], r[key]), (rep, k, key)
    del batch


def test_run_stamps_cover_every_unit(rrc):
    n, U, T = 16, 6, 512
    v, g = make_units(n, U, T)
    plan, _ = _plan(rrc, n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    ref = plan.run(vd, gains_in=gin, mode="pipelined")
    for mode in ("pipelined", "selfcal"):
        out = plan.alloc_outputs(DEV)
        out["stamps"] = torch.full((1 + U,), -1, dtype=torch.int64, device=DEV)
        plan.run(vd, gains_in=gin, mode=mode, out=out)
        torch.cuda.synchronize()
        st = out["stamps"].cpu().numpy()
        assert st[0] > 0 and np.all(st[1:] >= st[0]), (mode, st)
        if mode == "pipelined":
            for key in ("vunique", "gains", "chisq"):
                assert torch.equal(out[key], ref[key]), key
    hz = rrc.wall_clock_hz()
    assert 1e6 <= hz <= 1e10
    lat = (st[1:] - st[0]) / hz
    assert np.all(lat < 10.0)


def test_pipelined_gains_fed_back_in_place(rrc):
    # the real-time loop passing one buffer as both gains_in and gains_out:
    # the FFT-correlator must still apply the old gains (it reads a copy)
    n, U, T = 16, 16, 2048
    v, g = make_units(n, U, T)
    plan, _ = _plan(rrc, n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    g32 = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    ref = plan.run(vd, gains_in=g32.clone(), mode="pipelined")
    out = plan.alloc_outputs(DEV)
    out["gains"] = g32.clone()
    plan.run(vd, gains_in=out["gains"], mode="pipelined", out=out)
    torch.cuda.synchronize()
    for key in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq"):
        assert torch.equal(out[key], ref[key]), key


@pytest.mark.parametrize("dtype", ["c64", "ci4"])
def test_branch_orders_give_identical_results(rrc, dtype):
    n, U, T = 16, 4, 1024
    if dtype == "ci4":
        b, _, _, g = make_ci4_units(n, U, T)
        vd = torch.from_numpy(b).to(DEV)
    else:
        v, g = make_units(n, U, T)
        vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    plan, _ = _plan(rrc, n, U, T, dtype=dtype)
    a = plan.run(vd, gains_in=gin, mode="pipelined")
    for order in ("fft_first", "serial"):
        plan.set_order(order)
        b2 = plan.run(vd, gains_in=gin, mode="pipelined", out=plan.alloc_outputs(DEV))
        torch.cuda.synchronize()
        for key in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "niter", "status"):
            assert torch.equal(a[key], b2[key]), (order, key)


@pytest.mark.parametrize("dtype", ["c64", "ci4"])
def test_tuner_choice_cached_and_results_unchanged(rrc, dtype, tmp_path):
    n, U, T = 16, 8, 1024
    if dtype == "ci4":
        b, re, im, g = make_ci4_units(n, U, T)
        vd = torch.from_numpy(b).to(DEV)
        v = re.astype(np.complex128) + 1j * im.astype(np.complex128)
    else:
        v, g = make_units(n, U, T)
        vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    plan, _ = _plan(rrc, n, U, T, dtype=dtype)
    ref = plan.run(vd, gains_in=gin, mode="pipelined")
    cache = str(tmp_path / "tune.txt")
    t1 = plan.tune(vd, gin, cache_path=cache)
    assert t1["from_cache"] == 0 and t1["ms_per_run"] > 0
    got = plan.run(vd, gains_in=gin, mode="pipelined", out=plan.alloc_outputs(DEV))
    torch.cuda.synchronize()
    for key in ("vred", "gains", "vmodel", "chisq", "niter", "status"):
        assert torch.equal(got[key], ref[key]), key
    # another time chunking sums V^unique's partial grids in another order:
    # the tuned result is held to the oracle at the V^unique tolerance
    vu = got["vunique"].cpu().numpy()
    for u in range(U):
        want, _ = oracle_vunique(v[u], g[u].astype(np.complex64).astype(np.complex128), n)
        assert rel_l2(vu[u], want) <= TOL_VUNIQUE
    plan2, _ = _plan(rrc, n, U, T, dtype=dtype)
    t2 = plan2.tune(vd, gin, cache_path=cache)
    assert t2["from_cache"] == 1
    for k in ("fft_chunk_factor", "order", "xengine", "fft_size"):
        assert t2[k] == t1[k], k
    print(f"{dtype}: tuned {t1}")


def test_tuner_weighs_fft_sizes_and_keeps_results(rrc, tmp_path):
    # a 24 x 24 grid: the tuner times the 48- and the 64-point transform
    n, U, T = 24, 4, 1024
    v, g = make_units(n, U, T)
    vd = torch.from_numpy(v).to(DEV)
    gin = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    plan, _ = _plan(rrc, n, U, T)
    ref = plan.run(vd, gains_in=gin, mode="pipelined")
    t1 = plan.tune(vd, gin, cache_path=str(tmp_path / "tune.txt"))
    assert t1["fft_size"] in (48, 64)
    got = plan.run(vd, gains_in=gin, mode="pipelined", out=plan.alloc_outputs(DEV))
    torch.cuda.synchronize()
    for key in ("vred", "gains", "vmodel", "chisq", "niter", "status"):
        assert torch.equal(got[key], ref[key]), key
    vu = got["vunique"].cpu().numpy()
    for u in range(U):
        want, _ = oracle_vunique(v[u], g[u].astype(np.complex64).astype(np.complex128), n)
        assert rel_l2(vu[u], want) <= TOL_VUNIQUE
    print(f"n=24: tuned {t1}")
