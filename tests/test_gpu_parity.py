"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import redcal as OR
from tests.gpu_util import (TOL_GAINS, TOL_VUNIQUE, TOL_XENG, linearized_ls_reference, make_ci4_units,
                            make_units, oracle_solve, oracle_vunique, pairs_of, rel_l2)

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


@pytest.mark.parametrize("n,U,T", [(8, 2, 300), (8, 3, 301), (12, 2, 130), (16, 1, 1027), (16, 2, 1024),
                                   (64, 2, 4096), (4, 1, 1), (64, 1, 1)])
def test_xengine_ci4_bit_exact(rrc, n, U, T):
    b, re, im, _ = make_ci4_units(n, U, T)
    plan, types = _plan(rrc, n, U, T, dtype="ci4")
    vr = plan.xengine(torch.from_numpy(b).to(DEV)).cpu().numpy().astype(np.int64)
    pairs, _ = pairs_of(n, types)
    for u in range(U):
        ref = OC.xengine_int(re[u], im[u], pairs)
        assert np.array_equal(vr[u], ref), f"unit {u}: {np.sum(vr[u] != ref)} mismatches"


@pytest.mark.parametrize("n,T", [(8, 259), (16, 1024)])
def test_xengine_ci4_full_nibble_range(rrc, n, T):
    # every byte value, so both nibbles take -8 .. 7 (the -8 products included)
    from synthdata.generate import unpack_ci4
    rng = np.random.default_rng(17)
    b = rng.integers(0, 256, size=(2, T, n * n), dtype=np.uint8)
    b[:, :4, :] = 0x88                       # (-8, -8) at the start of each unit
    plan, types = _plan(rrc, n, 2, T, dtype="ci4")
    vr = plan.xengine(torch.from_numpy(b).to(DEV)).cpu().numpy().astype(np.int64)
    pairs, _ = pairs_of(n, types)
    for u in range(2):
        re, im = unpack_ci4(b[u])
        ref = OC.xengine_int(re, im, pairs)
        assert np.array_equal(vr[u], ref), f"unit {u}: {np.sum(vr[u] != ref)} mismatches"


# ----------------------------------------------------------------------- (a5)

@pytest.mark.parametrize("n,U,T,snr", [(8, 1, 256, 10.0), (16, 4, 1024, 10.0), (32, 2, 2048, 5.0)])
def test_solve_matches_oracle(rrc, n, U, T, snr):
    v, _ = make_units(n, U, T, snr=snr)
    plan, types = _plan(rrc, n, U, T)
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    out = plan.solve(vr_d)
    vr = vr_d.cpu().numpy()
    for u in range(U):
        ref = oracle_solve(vr[u].astype(np.complex128), n, types)
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        gerr = np.max(np.abs(g - ref["g"]) / np.abs(ref["g"]))
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
    # complex64: the solve must return the least-squares answer for the
    # rounded data (first-order reference from the injected truth) up to the
    # four degeneracies, at the sizes of the uneven-batch and 4-bit
    # workloads (2 and 4 antennas per work-item, up to 16 types, the whole
    # unit state in LDS).
    U = 2
    types, _ = rrc.select_subset(n)
    pos = OG.square_positions(n)
    pairs, tix = pairs_of(n, types)
    rng = np.random.default_rng(1000 + n)
    vred = np.empty((U, len(pairs)), np.complex64)
    truth = []
    for u in range(U):
        g = (1 + 0.05 * rng.standard_normal(n * n)) * np.exp(1j * rng.uniform(-np.pi, np.pi, n * n))
        vm = (0.2 + rng.random(len(types))) * np.exp(1j * rng.uniform(-np.pi, np.pi, len(types)))
        vred[u] = OR.model_vis(g, vm, pairs, tix).astype(np.complex64)
        gl, vl = linearized_ls_reference(vred[u], g, vm, pairs, tix, len(types))
        truth.append(OR.fix_refant(gl, vl, pos, types))
    plan = rrc.Plan(n, types, U, 64)
    out = plan.solve(torch.from_numpy(vred).to(DEV))
    for u in range(U):
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        gerr = np.max(np.abs(g - truth[u][0]) / np.abs(truth[u][0]))
        print(f"n={n} unit {u}: gains {gerr:.2e} niter {int(out['niter'][u])} status {int(out['status'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS


def test_solve_n24_matches_oracle(rrc):
    # a grid between the power-of-two sizes (ragged last wave, 7 types)
    n, U, T = 24, 2, 512
    v, _ = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    out = plan.solve(vr_d)
    vr = vr_d.cpu().numpy()
    for u in range(U):
        ref = oracle_solve(vr[u].astype(np.complex128), n, types)
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        gerr = np.max(np.abs(g - ref["g"]) / np.abs(ref["g"]))
        print(f"n={n} unit {u}: gains {gerr:.2e} niter {int(out['niter'][u])}")
        assert int(out["status"][u]) == 0
        assert gerr <= TOL_GAINS


def test_solve_ci4_matches_oracle(rrc):
    n, U, T = 16, 2, 1024
    b, re, im, _ = make_ci4_units(n, U, T)
    plan, types = _plan(rrc, n, U, T, dtype="ci4")
    vr_d = plan.xengine(torch.from_numpy(b).to(DEV))
    out = plan.solve(vr_d)
    vr = vr_d.cpu().numpy().astype(np.float64)
    for u in range(U):
        ref = oracle_solve(vr[u, :, 0] + 1j * vr[u, :, 1], n, types)
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(g - ref["g"]) / np.abs(ref["g"])) <= TOL_GAINS


def test_solve_from_gains_and_match_mode(rrc):
    n, U, T = 16, 2, 1024
    v, gtrue = make_units(n, U, T)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T, init_mode="gains", degen_mode="match")
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    gin = torch.from_numpy(gtrue.astype(np.complex64)).to(DEV)
    out = plan.solve(vr_d, gains_in=gin, gains_ref=gin)
    vr = vr_d.cpu().numpy().astype(np.complex128)
    for u in range(U):
        gref = gtrue[u].astype(np.complex64).astype(np.complex128)
        # matching phases is only well posed near the reference: start both there
        pairs, tix = pairs_of(n, types)
        ref = oracle_solve(vr[u], n, types, fix="match", g_ref=gref,
                           init=(gref, OR.group_mean(vr[u], gref, pairs, tix, len(types))))
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(g - ref["g"]) / np.abs(ref["g"])) <= TOL_GAINS
        assert int(out["status"][u]) == 0


def test_solve_nonfinite_unit_is_flagged(rrc):
    n, U, T = 8, 2, 128
    v, _ = make_units(n, U, T)
    v[1, 5, 7] = np.nan
    plan, _ = _plan(rrc, n, U, T)
    out = plan.run(torch.from_numpy(v).to(DEV), mode="selfcal")
    st = out["status"].cpu().numpy()
    assert st[0] == 0 and st[1] == 2


# ----------------------------------------------------------------------- (a6)

def test_chisq_and_adjoint_match_oracle(rrc):
    n, U, T = 16, 3, 512
    v, gtrue = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    pairs, tix = pairs_of(n, types)
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    rng = np.random.default_rng(3)
    g = (gtrue * (1 + 0.03 * (rng.standard_normal(gtrue.shape) + 1j * rng.standard_normal(gtrue.shape)))).astype(np.complex64)
    vm = np.stack([OR.group_mean(vr_d[u].cpu().numpy().astype(np.complex128), gtrue[u], pairs, tix, len(types))
                   for u in range(U)]).astype(np.complex64)
    gd, vmd = torch.from_numpy(g).to(DEV), torch.from_numpy(vm).to(DEV)
    c = plan.chisq_fwd(gd, vmd, vr_d).cpu().numpy()
    gg, gv, dg, dv = [x.cpu().numpy() for x in plan.chisq_adj(gd, vmd, vr_d)]
    vr = vr_d.cpu().numpy()
    for u in range(U):
        g64, v64, r64 = g[u].astype(np.complex128), vm[u].astype(np.complex128), vr[u].astype(np.complex128)
        cref = OR.chisq(r64, g64, v64, pairs, tix)
        assert abs(c[u] - cref) <= 1e-5 * cref
        rg, rv = OR.wirtinger_grad(r64, g64, v64, pairs, tix)
        hg, hv = OR.jhj_diag(g64, v64, pairs, tix)
        sc = np.max(np.abs(2 * rg))
        assert np.max(np.abs(gg[u] - 2 * rg)) <= 1e-5 * sc
        assert np.max(np.abs(gv[u] - 2 * rv)) <= 1e-5 * np.max(np.abs(2 * rv))
        assert np.max(np.abs(dg[u] - hg) / hg) <= 1e-5
        assert np.max(np.abs(dv[u] - hv) / hv) <= 1e-5


def test_adjoint_matches_central_finite_differences(rrc):
    # chi^2 is quadratic in each single complex parameter (no pair has
    # i = j), so central differences of the FP64 chi^2 with step 1e-3 are
    # exact up to rounding: d chi2/d Re z + i d chi2/d Im z = 2 d chi2/d conj(z),
    # which is what rrc_chisq_adj returns
    n, U, T = 8, 1, 256
    v, gtrue = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    pairs, tix = pairs_of(n, types)
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    vr = vr_d.cpu().numpy()[0].astype(np.complex128)
    rng = np.random.default_rng(11)
    g = (gtrue[0] * (1 + 0.02 * (rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)))).astype(np.complex64)
    vm = OR.group_mean(vr, gtrue[0], pairs, tix, len(types)).astype(np.complex64)
    gg, gv, _, _ = plan.chisq_adj(torch.from_numpy(g[None]).to(DEV), torch.from_numpy(vm[None]).to(DEV), vr_d)
    gg, gv = gg.cpu().numpy()[0], gv.cpu().numpy()[0]
    g64, v64 = g.astype(np.complex128), vm.astype(np.complex128)
    h = 1e-3

    def fd(vec_g, vec_v, which, k):
        out = 0j
        for part, unit in ((0, 1.0), (1, 1j)):
            gp, gm, vp, vmn = vec_g.copy(), vec_g.copy(), vec_v.copy(), vec_v.copy()
            if which == "g":
                gp[k] += h * unit
                gm[k] -= h * unit
            else:
                vp[k] += h * unit
                vmn[k] -= h * unit
            d = (OR.chisq(vr, gp, vp, pairs, tix) - OR.chisq(vr, gm, vmn, pairs, tix)) / (2 * h)
            out += d * (1 if part == 0 else 1j)
        return out

    sc_g = np.max(np.abs(gg))
    for k in rng.choice(n * n, size=8, replace=False):
        assert abs(gg[k] - fd(g64, v64, "g", k)) <= 1e-5 * sc_g, k
    sc_v = np.max(np.abs(gv))
    for k in range(len(types)):
        assert abs(gv[k] - fd(g64, v64, "v", k)) <= 1e-5 * sc_v, k


def test_chisq_autograd_function(rrc):
    n, U, T = 8, 2, 256
    v, gtrue = make_units(n, U, T)
    plan, types = _plan(rrc, n, U, T)
    vr_d = plan.xengine(torch.from_numpy(v).to(DEV))
    g = torch.from_numpy(gtrue.astype(np.complex64)).to(DEV).requires_grad_(True)
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
    # end to end against the oracle: gains from the GPU V^reduced, V^unique with the GPU gains
    for u in range(U):
        ref = oracle_solve(b["vred"][u].cpu().numpy().astype(np.complex128), n, types)
        g = b["gains"][u].cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(g - ref["g"]) / np.abs(ref["g"])) <= TOL_GAINS
        vref, _ = oracle_vunique(v[u], g, n)
        assert rel_l2(b["vunique"][u].cpu().numpy(), vref) <= TOL_VUNIQUE


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


@pytest.mark.skip(reason="capturing the batch into a HIP graph ended the test process with a host "
                         "segmentation fault inside rrc_batch_run; no cause was found in this code, so "
                         "the graph path was removed and the batch launches its branches eagerly")
def test_batch_graph_matches_eager_runs(rrc):
    plans, volts, gins = _batch_inputs(rrc)
    batch = rrc.Batch(plans)
    outs = [p.alloc_outputs(DEV) for p in plans]
    ref = [p.run(v, gains_in=gi, mode="pipelined") for p, v, gi in zip(plans, volts, gins)]
    for rep in range(3):
        batch.run(volts, gins, outs, mode="pipelined")
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o["gains"], r["gains"])
