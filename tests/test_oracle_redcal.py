"""Pins for oracle.redcal: exact recovery of noise-free model data, the
Wirtinger gradient against finite differences (exact: chi^2 is quadratic in
every single parameter), stationarity, two independent solvers agreeing, the
DoF count against the Jacobian's null space, the degeneracy fixes, and the
pair-by-pair normal equations against the dense Jacobian (whose columns are
pinned by exact central differences of the model) and the minimum-norm
least-squares steps against numpy's pseudo-inverse solution."""
import numpy as np
import pytest

from oracle import correlator as C
from oracle import geometry as G
from oracle import redcal as R


def _problem(n, types, seed, noise=0.0, nt=None):
    rng = np.random.default_rng(seed)
    pos = G.square_positions(n)
    pairs, tix = G.group_pairs(pos, types)
    g = (1 + 0.05 * rng.standard_normal(n * n)) * np.exp(1j * rng.uniform(-np.pi, np.pi, n * n))
    vm = (0.5 + rng.uniform(0, 0.5, len(types))) * np.exp(1j * rng.uniform(-np.pi, np.pi, len(types)))
    vred = R.model_vis(g, vm, pairs, tix)
    if noise:
        vred = vred + noise * (rng.standard_normal(len(vred)) + 1j * rng.standard_normal(len(vred)))
    return pos, pairs, tix, g, vm, vred


@pytest.mark.parametrize("n,k", [(4, 3), (6, 5), (8, 5), (10, 7)])
def test_noise_free_recovery(n, k):
    types = G.square_types(n)[0][:k]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=n)
    out = R.calibrate(vred, pos, types, pairs, tix)
    assert out["converged"]
    assert out["chisq"] < 1e-20
    gt, vt = R.fix_refant(g, vm, pos, types)
    assert np.max(np.abs(out["g"] - gt)) < 1e-12
    assert np.max(np.abs(out["vm"] - vt)) < 1e-12


def test_gradient_central_differences():
    n = 5
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=11, noise=0.1)
    rng = np.random.default_rng(12)
    g = g * (1 + 0.05 * (rng.standard_normal(len(g)) + 1j * rng.standard_normal(len(g))))
    dg, dv = R.wirtinger_grad(vred, g, vm, pairs, tix)
    h = 1e-3

    def f(gg, vv):
        return R.chisq(vred, gg, vv, pairs, tix)

    for k in range(len(g)):
        for unit, part in ((1.0, "re"), (1j, "im")):
            gp, gm = g.copy(), g.copy()
            gp[k] += h * unit
            gm[k] -= h * unit
            fd = (f(gp, vm) - f(gm, vm)) / (2 * h)
            an = 2 * (dg[k].real if part == "re" else dg[k].imag)   # 2 d/dconj(z) = d/dRe + i d/dIm
            assert abs(fd - an) <= 1e-9 * (1 + abs(an))
    for k in range(len(vm)):
        for unit, part in ((1.0, "re"), (1j, "im")):
            vp, vn = vm.copy(), vm.copy()
            vp[k] += h * unit
            vn[k] -= h * unit
            fd = (f(g, vp) - f(g, vn)) / (2 * h)
            an = 2 * (dv[k].real if part == "re" else dv[k].imag)
            assert abs(fd - an) <= 1e-9 * (1 + abs(an))


def test_jhj_diag_matches_dense_jacobian():
    n = 4
    types = G.square_types(n)[0][:4]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=13)
    hg, hv = R.jhj_diag(g, vm, pairs, tix)
    jr = R.jacobian_real(g, vm, pairs, tix)
    d = np.sum(jr ** 2, axis=0)
    nant, nt = len(g), len(vm)
    assert np.allclose(d[:nant], hg, rtol=1e-13)
    assert np.allclose(d[nant:2 * nant], hg, rtol=1e-13)
    assert np.allclose(d[2 * nant:2 * nant + nt], hv, rtol=1e-13)


def test_stationary_and_solvers_agree():
    n = 5
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=14, noise=0.02)
    a = R.calibrate(vred, pos, types, pairs, tix, solver="lincal", tol=1e-13)
    dg, dv = R.wirtinger_grad(vred, a["g"], a["vm"], pairs, tix)
    assert np.max(np.abs(np.concatenate([dg, dv]))) < 1e-10
    b = R.calibrate(vred, pos, types, pairs, tix, solver="omnical", tol=1e-13)
    assert b["converged"]
    assert np.max(np.abs(a["g"] - b["g"])) < 1e-8
    assert abs(a["chisq"] - b["chisq"]) < 1e-12


def test_degenerate_directions_are_null():
    n = 6
    types = G.square_types(n)[0][:6]
    pos, pairs, tix, g, vm, _ = _problem(n, types, seed=15)
    jr = R.jacobian_real(g, vm, pairs, tix)
    z = R._real(*R.degenerate_directions(g, vm, pos, types))
    assert np.max(np.abs(jr @ z.T)) < 1e-12
    # the Jacobian's null space has exactly these four directions (Sec. 5.2)
    sv = np.linalg.svd(jr, compute_uv=False)
    assert np.sum(sv < 1e-9 * sv[0]) == 4


@pytest.mark.parametrize("n,k", [(5, 5), (8, 6)])
def test_dof_equals_real_dof_over_two(n, k):
    types = G.square_types(n)[0][:k]
    pos, pairs, tix, g, vm, _ = _problem(n, types, seed=16)
    jr = R.jacobian_real(g, vm, pairs, tix)
    rank = np.linalg.matrix_rank(jr)
    real_dof = 2 * len(pairs) - rank            # real equations minus identifiable parameters
    assert 2 * R.dof(len(pairs), n * n, len(types)) == real_dof


def test_fix_refant_properties():
    n = 6
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=17, noise=0.05)
    g2, v2 = R.fix_refant(g, vm, pos, types)
    assert np.allclose(R.model_vis(g2, v2, pairs, tix), R.model_vis(g, vm, pairs, tix), atol=1e-14)
    assert abs(np.sum(np.log(np.abs(g2)))) < 1e-12
    for a in (0, 1, n):
        assert abs(np.angle(g2[a])) < 1e-14 and g2[a].real > 0
    g3, v3 = R.fix_refant(g2, v2, pos, types)
    assert np.max(np.abs(g3 - g2)) < 1e-14
    # any degenerate transform of the input lands on the same representative
    lam, th, kx, ky = 1.3, 0.7, 2.9, -1.1
    gd = lam * g * np.exp(1j * (th + kx * pos[:, 0] + ky * pos[:, 1]))
    d = np.asarray(types, float)
    vd = vm / lam ** 2 * np.exp(-1j * (kx * d[:, 0] + ky * d[:, 1]))
    g4, v4 = R.fix_refant(gd, vd, pos, types)
    assert np.max(np.abs(g4 - g2)) < 1e-12 and np.max(np.abs(v4 - v2)) < 1e-12


def test_fix_match_restores_reference():
    n = 5
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, _ = _problem(n, types, seed=18)
    d = np.asarray(types, float)
    gd = 0.8 * g * np.exp(1j * (0.3 + 0.2 * pos[:, 0] - 0.4 * pos[:, 1]))
    vd = vm / 0.64 * np.exp(-1j * (0.2 * d[:, 0] - 0.4 * d[:, 1]))
    g2, v2 = R.fix_match(gd, vd, g, pos, types)
    assert np.max(np.abs(g2 - g)) < 1e-12 and np.max(np.abs(v2 - vm)) < 1e-12


def test_logcal_amplitude_noise_free():
    n = 6
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=19)
    amp, vamp = R.logcal_amplitude(vred, pairs, tix, n * n, len(types))
    # equal up to the amplitude degeneracy |g| -> l |g|, |V| -> |V| / l^2
    lam = np.exp(np.mean(np.log(amp)) - np.mean(np.log(np.abs(g))))
    assert np.allclose(amp / lam, np.abs(g), rtol=1e-12)
    assert np.allclose(vamp * lam ** 2, np.abs(vm), rtol=1e-12)


def test_firstcal_noise_free_is_exact_up_to_degeneracy():
    n = 7
    types = G.square_types(n)[0][:6]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=20)
    g0, v0 = R.firstcal(vred, pos, types, pairs, tix)
    assert R.chisq(vred, g0, v0, pairs, tix) < 1e-20


def test_voltage_level_end_to_end_basin():
    # Voltage-level data: the solver from the defined starting point and from
    # the true gains must reach the same minimum, with chi^2 below the truth's.
    from synthdata import unit_gains, unit_voltages
    n, m, t = 8, 16, 256
    g = unit_gains(0, 0, n, 1, False)[0]
    v = unit_voltages(0, 0, 0, n, m, t, 10.0, g)
    pos = G.square_positions(n)
    types = G.select_subset_square(n)
    pairs, tix = G.group_pairs(pos, types)
    vred = C.xengine(C.fx_correlate(v), pairs)
    a = R.calibrate(vred, pos, types, pairs, tix)
    b = R.calibrate(vred, pos, types, pairs, tix, init=(g, R.group_mean(vred, g, pairs, tix, len(types))))
    assert a["converged"] and b["converged"]
    assert np.max(np.abs(a["g"] - b["g"])) < 1e-9
    assert a["chisq"] <= R.chisq(vred, g, R.group_mean(vred, g, pairs, tix, len(types)), pairs, tix)


# ------------------------------------------------ normal equations per pair

def test_jacobian_columns_are_central_differences():
    # the model g_i conj(g_j) V_alpha is linear in each single real unknown,
    # so central differences of it are exact up to rounding
    n = 4
    types = G.square_types(n)[0][:4]
    pos, pairs, tix, g, vm, _ = _problem(n, types, seed=21)
    jr = R.jacobian_real(g, vm, pairs, tix)
    nant, nt = len(g), len(vm)
    h = 1e-3
    for col in range(2 * (nant + nt)):
        x = np.concatenate([g.real, g.imag, vm.real, vm.imag])
        xp, xm = x.copy(), x.copy()
        xp[col] += h
        xm[col] -= h

        def mv(xx):
            gg = xx[:nant] + 1j * xx[nant:2 * nant]
            vv = xx[2 * nant:2 * nant + nt] + 1j * xx[2 * nant + nt:]
            m = R.model_vis(gg, vv, pairs, tix)
            return np.concatenate([m.real, m.imag])

        fd = (mv(xp) - mv(xm)) / (2 * h)
        assert np.max(np.abs(fd - jr[:, col])) < 1e-11


@pytest.mark.parametrize("n,k", [(4, 3), (6, 5), (10, 7)])
def test_normal_equations_per_pair_match_dense_jacobian(n, k):
    types = G.square_types(n)[0][:k]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=30 + n, noise=0.1)
    h, rhs = R.normal_equations(vred, g, vm, pairs, tix)
    jr = R.jacobian_real(g, vm, pairs, tix)
    r = vred - R.model_vis(g, vm, pairs, tix)
    hd = jr.T @ jr
    assert np.max(np.abs(h.toarray() - hd)) <= 1e-12 * np.max(np.abs(hd))
    rd = jr.T @ np.concatenate([r.real, r.imag])
    assert np.max(np.abs(rhs - rd)) <= 1e-12 * np.max(np.abs(rd))


@pytest.mark.parametrize("n,k", [(5, 5), (8, 6)])
def test_gauss_newton_step_is_the_minimum_norm_least_squares_step(n, k):
    # the step lincal takes equals the pseudo-inverse solution of the dense
    # linearised system J dx = r
    types = G.square_types(n)[0][:k]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=40 + n, noise=0.1)
    g = g * (1 + 0.05 * np.random.default_rng(n).standard_normal(len(g)))
    h, rhs = R.normal_equations(vred, g, vm, pairs, tix)
    dx = R.min_norm_solve(h, rhs, R._real(*R.degenerate_directions(g, vm, pos, types)))
    jr = R.jacobian_real(g, vm, pairs, tix)
    r = vred - R.model_vis(g, vm, pairs, tix)
    ref = np.linalg.lstsq(jr, np.concatenate([r.real, r.imag]), rcond=1e-10)[0]
    assert np.max(np.abs(dx - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_logcal_amplitude_is_the_minimum_norm_least_squares_fit():
    n = 6
    types = G.square_types(n)[0][:5]
    pos, pairs, tix, g, vm, vred = _problem(n, types, seed=50, noise=0.1)
    amp, vamp = R.logcal_amplitude(vred, pairs, tix, n * n, len(types))
    a = np.zeros((len(pairs), n * n + len(types)))
    rows = np.arange(len(pairs))
    a[rows, pairs[:, 0]] += 1.0
    a[rows, pairs[:, 1]] += 1.0
    a[rows, n * n + tix] += 1.0
    x = np.linalg.lstsq(a, np.log(np.abs(vred)), rcond=None)[0]
    assert np.max(np.abs(np.log(amp) - x[:n * n])) < 1e-12
    assert np.max(np.abs(np.log(vamp) - x[n * n:])) < 1e-12


def test_refant_fix_on_a_hexagonal_array():
    # Sec. 5.2 reference antennas on a lattice whose grid corner is empty:
    # the first antenna in raster order and its +x, +y neighbours become
    # real and positive, mean ln|g| becomes 0, and every model visibility
    # g_i conj(g_j) V_alpha is unchanged (the fix moves along the
    # degeneracies only)
    _, _, pos = G.hex_grid(4)
    types = [(1, 0), (-1, 1), (0, 1), (1, 1)]
    pairs, tix = G.group_pairs(pos, types)
    rng = np.random.default_rng(3)
    g = (1 + 0.3 * rng.standard_normal(len(pos))) * np.exp(1j * rng.uniform(-3, 3, len(pos)))
    vm = rng.standard_normal(len(types)) + 1j * rng.standard_normal(len(types))
    g2, vm2 = R.fix_refant(g, vm, pos, types)
    idx = G.PositionIndex(pos)
    a0 = idx.lut[3 - idx.lo[0], 0 - idx.lo[1]]
    ax = idx.lut[4 - idx.lo[0], 0 - idx.lo[1]]
    ay = idx.lut[3 - idx.lo[0], 1 - idx.lo[1]]
    assert (tuple(pos[a0]), tuple(pos[ax]), tuple(pos[ay])) == ((3, 0), (4, 0), (3, 1))
    for a in (a0, ax, ay):
        assert abs(g2[a].imag) < 1e-12 and g2[a].real > 0
    assert abs(np.mean(np.log(np.abs(g2)))) < 1e-12
    np.testing.assert_allclose(R.model_vis(g2, vm2, pairs, tix), R.model_vis(g, vm, pairs, tix),
                               rtol=1e-12, atol=1e-12)
