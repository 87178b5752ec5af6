"""Redundant-baseline calibration on a (reduced) set of visibilities, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Sec. 2, eq. redcal): V_b = g_i conj(g_j) V_alpha + n_b for each
selected pair b = (i, j) of type alpha (r_i - r_j = d_alpha).  Unknowns are
the N antenna gains g and the K model visibilities V_alpha.  The fit
minimises chi^2 = sum_b |V_b - g_i conj(g_j) V_alpha|^2 (eq. redchi with
uniform noise, which is what eq. noisecov assumes), with
DoF = N_obs - N - N_ubl + 2 (eq. dof).

Solvers
-------
* `logcal_amplitude`: the real part of eq. logcal, solved by linear least
  squares (a starting point only: it is noise-biased, Sec. 2).
* `firstcal`: logcal amplitudes plus phases propagated along the (1,0) and
  (0,1) redundant groups (a definition of this library; the paper does not
  say how its solver was started).
* `lincal`: Gauss-Newton on the Taylor-expanded model (the "Taylor
  expansion" linearisation of Sec. 2): FP64 normal equations of the
  real-stacked Jacobian, assembled pair by pair from each pair's 6 x 6
  block, solved for the minimum-norm step (orthogonal to the four
  degenerate directions of Sec. 5.2) by a sparse direct solve of the
  bordered system, iterated until ||dx|| / ||x|| < 1e-10 (Sec. 3).
* `omnical`: per-parameter least-squares updates blended with a damping
  factor of 0.3 (the paper's omnical settings, Sec. 3; its update rule is
  only cited there, this is the reading used here).
* `fix_refant` / `fix_match`: remove the four degeneracies (Sec. 5.2).
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np

from .geometry import PositionIndex


# --------------------------------------------------------------------------- model

def model_vis(g, vm, pairs, tix):
    """g_i conj(g_j) V_alpha for each selected pair (eq. redcal, noise-free)."""
    return g[pairs[:, 0]] * np.conj(g[pairs[:, 1]]) * vm[tix]


def chisq(vred, g, vm, pairs, tix) -> float:
    """Unweighted chi^2 of eq. redchi (sigma_ij = 1)."""
    r = vred - model_vis(g, vm, pairs, tix)
    return float(np.sum(np.abs(r) ** 2))


def dof(n_obs: int, n_ant: int, n_ubl: int) -> int:
    """Degrees of freedom of eq. dof: N_obs - N - N_ubl + 2."""
    return n_obs - n_ant - n_ubl + 2


def wirtinger_grad(vred, g, vm, pairs, tix):
    """d chi^2 / d conj(g_i) and d chi^2 / d conj(V_alpha).

    With r_b = V_b - g_i conj(g_j) V_alpha:
      d/d conj(g_i)   = - sum_{b=(i,j)} r_b g_j conj(V_alpha)
                        - sum_{b=(k,i)} conj(r_b) g_k V_beta
      d/d conj(V_a)   = - sum_{b in a} r_b conj(g_i) g_j
    """
    i, j = pairs[:, 0], pairs[:, 1]
    r = vred - model_vis(g, vm, pairs, tix)
    dg = np.zeros(len(g), dtype=np.complex128)
    np.add.at(dg, i, -r * g[j] * np.conj(vm[tix]))
    np.add.at(dg, j, -np.conj(r) * g[i] * vm[tix])
    dv = np.zeros(len(vm), dtype=np.complex128)
    np.add.at(dv, tix, -r * np.conj(g[i]) * g[j])
    return dg, dv


def jhj_diag(g, vm, pairs, tix):
    """Diagonal of J^H J: sum over a parameter's pairs of |d model / d param|^2."""
    i, j = pairs[:, 0], pairs[:, 1]
    hg = np.zeros(len(g))
    np.add.at(hg, i, np.abs(g[j] * vm[tix]) ** 2)
    np.add.at(hg, j, np.abs(g[i] * vm[tix]) ** 2)
    hv = np.zeros(len(vm))
    np.add.at(hv, tix, np.abs(g[i] * g[j]) ** 2)
    return hg, hv


# ---------------------------------------------------------------- starting point

def logcal_amplitude(vred, pairs, tix, n_ant: int, n_types: int):
    """Real part of eq. logcal: ln|V_b| = eta_i + eta_j + A_alpha, least squares.

    Returns (|g| [N], |V| [K]) from the minimum-norm solution.  The system
    A (one row per pair, ones at eta_i, eta_j and A_alpha) is singular along
    the amplitude degeneracy (eta += c, A -= 2c, Sec. 5.2); its normal
    equations are solved orthogonally to that direction (`min_norm_solve`).
    """
    import scipy.sparse as sp
    npair = len(pairs)
    rows = np.repeat(np.arange(npair), 3)
    cols = np.stack([pairs[:, 0], pairs[:, 1], n_ant + tix], axis=1).ravel()
    a = sp.csr_matrix((np.ones(3 * npair), (rows, cols)), shape=(npair, n_ant + n_types))
    z = np.concatenate([np.ones(n_ant), -2.0 * np.ones(n_types)])[None, :]
    x = min_norm_solve((a.T @ a).tocsc(), a.T @ np.log(np.abs(vred)), z)
    return np.exp(x[:n_ant]), np.exp(x[n_ant:])


def firstcal(vred, pos, types: Sequence[Tuple[int, int]], pairs, tix):
    """Starting point: logcal amplitudes, chained phases, group-mean V_alpha.

    Phases: antenna (0,0) gets 0.  Along the bottom row, phi(x,0) =
    phi(x-1,0) + arg(V_b exp(-i psi_10)) for the (1,0) pair b =
    ((x,0),(x-1,0)), where psi_10 = arg of that group's pair at x = 1 (so
    that antenna (1,0) also gets phase 0).  Each column then climbs with the
    (0,1) pairs the same way, psi_01 being the arg of the pair
    ((0,1),(0,0)).  The selection must contain (1,0) and (0,1).
    """
    types = [tuple(t) for t in types]
    nant = len(pos)
    amp, _ = logcal_amplitude(vred, pairs, tix, nant, len(types))
    t10, t01 = types.index((1, 0)), types.index((0, 1))
    idx = PositionIndex(pos)
    lo = idx.lo
    rel = pos - lo
    nx, ny = idx.lut.shape
    v10 = np.full((nx, ny), np.nan + 0j)
    v01 = np.full((nx, ny), np.nan + 0j)
    sel = tix == t10
    v10[rel[pairs[sel, 0], 0], rel[pairs[sel, 0], 1]] = vred[sel]
    sel = tix == t01
    v01[rel[pairs[sel, 0], 0], rel[pairs[sel, 0], 1]] = vred[sel]
    psi10 = np.angle(v10[1, 0])
    psi01 = np.angle(v01[0, 1])
    phi = np.zeros((nx, ny))
    for x in range(1, nx):
        phi[x, 0] = phi[x - 1, 0] + np.angle(v10[x, 0] * np.exp(-1j * psi10))
    for y in range(1, ny):
        for x in range(nx):
            phi[x, y] = phi[x, y - 1] + np.angle(v01[x, y] * np.exp(-1j * psi01))
    g = amp * np.exp(1j * phi[rel[:, 0], rel[:, 1]])
    vm = group_mean(vred, g, pairs, tix, len(types))
    return g, vm


def group_mean(vred, g, pairs, tix, n_types: int):
    """V_alpha = mean over the group of V_b / (g_i conj(g_j))."""
    q = vred / (g[pairs[:, 0]] * np.conj(g[pairs[:, 1]]))
    s = np.zeros(n_types, dtype=np.complex128)
    np.add.at(s, tix, q)
    return s / np.bincount(tix, minlength=n_types)


# ------------------------------------------------------------------- degeneracies

def degenerate_directions(g, vm, pos, types):
    """Tangent vectors of the four degeneracies of Sec. 5.2 at (g, V).

    amplitude g -> l g, V -> V / l^2; phase g -> e^{i t} g; phase slopes
    g_i -> e^{i k.r_i} g_i, V_alpha -> e^{-i k.d_alpha} V_alpha.
    Returned as complex (dg [4, N], dv [4, K]).
    """
    d = np.asarray(types, dtype=float)
    r = np.asarray(pos, dtype=float)
    dg = np.stack([g, 1j * g, 1j * r[:, 0] * g, 1j * r[:, 1] * g])
    dv = np.stack([-2.0 * vm, 0.0 * vm, -1j * d[:, 0] * vm, -1j * d[:, 1] * vm])
    return dg, dv


def _real(dg, dv):
    return np.concatenate([dg.real, dg.imag, dv.real, dv.imag], axis=-1)


def jacobian_real(g, vm, pairs, tix):
    """Real-stacked Jacobian of the model, rows [Re; Im], cols [Re g, Im g, Re V, Im V]."""
    nant, nt, npair = len(g), len(vm), len(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    rows = np.arange(npair)
    jc = np.zeros((npair, 2 * (nant + nt)), dtype=np.complex128)
    a = np.conj(g[j]) * vm[tix]          # d m / d g_i
    b = g[i] * vm[tix]                   # d m / d conj(g_j)
    c = g[i] * np.conj(g[j])             # d m / d V_alpha
    jc[rows, i] += a
    jc[rows, nant + i] += 1j * a
    jc[rows, j] += b
    jc[rows, nant + j] += -1j * b
    jc[rows, 2 * nant + tix] += c
    jc[rows, 2 * nant + nt + tix] += 1j * c
    return np.vstack([jc.real, jc.imag])


def pair_columns(nant: int, nt: int, pairs, tix):
    """Columns of each pair's six real unknowns in [Re g, Im g, Re V, Im V] order.

    Pair b = (i, j) of type alpha depends on g_i, g_j and V_alpha only:
    columns (Re g_i, Im g_i, Re g_j, Im g_j, Re V_alpha, Im V_alpha).
    """
    i, j = pairs[:, 0], pairs[:, 1]
    return np.stack([i, nant + i, j, nant + j, 2 * nant + tix, 2 * nant + nt + tix], axis=1)


def pair_derivatives(g, vm, pairs, tix):
    """d model_b / d (each of the pair's six real unknowns), complex [P, 6].

    m_b = g_i conj(g_j) V_alpha, so with a = conj(g_j) V_alpha,
    b = g_i V_alpha, c = g_i conj(g_j):
    d/dRe g_i = a, d/dIm g_i = i a, d/dRe g_j = b, d/dIm g_j = -i b,
    d/dRe V = c, d/dIm V = i c.
    """
    i, j = pairs[:, 0], pairs[:, 1]
    a = np.conj(g[j]) * vm[tix]
    b = g[i] * vm[tix]
    c = g[i] * np.conj(g[j])
    return np.stack([a, 1j * a, b, -1j * b, c, 1j * c], axis=1)


def normal_equations(vred, g, vm, pairs, tix):
    """J^T J and J^T r of the real-stacked Gauss-Newton system, per pair.

    J is the real Jacobian of [Re m; Im m] (the Taylor expansion of eq.
    redcal about the current point, Sec. 2) and r = V^reduced - m.  Each
    pair touches six real unknowns, so J^T J is a sum of 6 x 6 blocks
    Re(conj(d_b) d_b^T) and J^T r a sum of 6-vectors Re(conj(d_b) r_b),
    d_b being the pair's row of complex derivatives.  Returns J^T J as a
    scipy sparse CSC matrix (entries of coincident columns summed) and
    J^T r as a dense vector, both FP64.
    """
    import scipy.sparse as sp
    nant, nt = len(g), len(vm)
    nv = 2 * (nant + nt)
    cols = pair_columns(nant, nt, pairs, tix)
    d = pair_derivatives(g, vm, pairs, tix)
    r = vred - model_vis(g, vm, pairs, tix)
    blk = np.real(np.conj(d)[:, :, None] * d[:, None, :])
    rows_ix = np.broadcast_to(cols[:, :, None], blk.shape).ravel()
    cols_ix = np.broadcast_to(cols[:, None, :], blk.shape).ravel()
    h = sp.coo_matrix((blk.ravel(), (rows_ix, cols_ix)), shape=(nv, nv)).tocsc()
    rhs = np.zeros(nv)
    np.add.at(rhs, cols, np.real(np.conj(d) * r[:, None]))
    return h, rhs


def min_norm_solve(h, rhs, z):
    """Minimum-norm solution of rank-deficient normal equations h dx = rhs.

    h = J^T J is singular exactly along the degenerate directions z
    ([k, n] rows, Sec. 5.2), and rhs = J^T r is orthogonal to them.  The
    solution orthogonal to z is the solution of the bordered system
    [[h, z^T], [z, 0]] [dx; lam] = [rhs; 0] (lam = 0 at the solution),
    solved by a sparse direct LU (minimum-degree ordering of h + h^T).
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    nv = h.shape[0]
    kkt = sp.bmat([[h, sp.csc_matrix(z.T)], [sp.csc_matrix(z), None]], format="csc")
    x = spl.spsolve(kkt, np.concatenate([rhs, np.zeros(len(z))]), permc_spec="MMD_AT_PLUS_A")
    return x[:nv]


def lincal(vred, pos, types, pairs, tix, g0, v0, tol: float = 1e-10, max_iter: int = 100):
    """Gauss-Newton on the Taylor-expanded redcal model, FP64.

    Each step is the minimum-norm least-squares solution of the linearised
    system, J^T J dx = J^T r with dx orthogonal to the four degenerate
    directions (`normal_equations`, `min_norm_solve`).  Stops when
    ||dx|| / ||x|| < tol.  Returns (g, V, n_iter, converged).
    """
    g = np.array(g0, dtype=np.complex128)
    vm = np.array(v0, dtype=np.complex128)
    nant, nt = len(g), len(vm)
    for it in range(1, max_iter + 1):
        h, rhs = normal_equations(vred, g, vm, pairs, tix)
        dx = min_norm_solve(h, rhs, _real(*degenerate_directions(g, vm, pos, types)))
        g = g + dx[:nant] + 1j * dx[nant:2 * nant]
        vm = vm + dx[2 * nant:2 * nant + nt] + 1j * dx[2 * nant + nt:]
        x = np.concatenate([g, vm])
        if np.linalg.norm(dx) / np.linalg.norm(np.concatenate([x.real, x.imag])) < tol:
            return g, vm, it, True
    return g, vm, max_iter, False


def omnical(vred, pairs, tix, g0, v0, gain: float = 0.3, tol: float = 1e-10,
            max_iter: int = 100000):
    """Damped simultaneous per-parameter least-squares updates.

    Holding all other parameters fixed, chi^2 is an exact quadratic in each
    single g_i or V_alpha (no pair has i = j), so its minimiser is
      g_i' = [sum_{(i,j)} V_b g_j conj(V_a) + sum_{(k,i)} conj(V_b) g_k V_b']
             / [sum |g_j V_a|^2 + sum |g_k V_b'|^2]
      V_a' = sum_{b in a} V_b conj(g_i) g_j / sum |g_i g_j|^2.
    All parameters move together, x <- x + gain (x' - x); the iteration stops
    when ||x_new - x|| / ||x_new|| < tol.  Returns (g, V, n_iter, converged).
    """
    g = np.array(g0, dtype=np.complex128)
    vm = np.array(v0, dtype=np.complex128)
    i, j = pairs[:, 0], pairs[:, 1]
    for it in range(1, max_iter + 1):
        num_g = np.zeros(len(g), dtype=np.complex128)
        np.add.at(num_g, i, vred * g[j] * np.conj(vm[tix]))
        np.add.at(num_g, j, np.conj(vred) * g[i] * vm[tix])
        num_v = np.zeros(len(vm), dtype=np.complex128)
        np.add.at(num_v, tix, vred * np.conj(g[i]) * g[j])
        hg, hv = jhj_diag(g, vm, pairs, tix)
        gn = g + gain * (num_g / hg - g)
        vn = vm + gain * (num_v / hv - vm)
        xo = np.concatenate([g, vm])
        xn = np.concatenate([gn, vn])
        g, vm = gn, vn
        if np.linalg.norm(xn - xo) / np.linalg.norm(xn) < tol:
            return g, vm, it, True
    return g, vm, max_iter, False


def _ref_antennas(pos):
    # Sec. 5.2 fixes the phase and the two phase slopes against reference
    # antennas without naming them: the first antenna in raster order (least
    # y, then least x) and its neighbours one step along x and along y.  On a
    # square grid these are (0,0), (1,0), (0,1).
    pos = np.asarray(pos, dtype=np.int64)
    a0 = int(np.lexsort((pos[:, 0], pos[:, 1]))[0])
    idx = PositionIndex(pos)
    r = pos[a0] - idx.lo
    ax = idx.lut[r[0] + 1, r[1]] if r[0] + 1 < idx.lut.shape[0] else -1
    ay = idx.lut[r[0], r[1] + 1] if r[1] + 1 < idx.lut.shape[1] else -1
    if min(ax, ay) < 0:
        raise ValueError("the first antenna's +x and +y neighbours must exist")
    return a0, int(ax), int(ay), pos - pos[a0]


def fix_refant(g, vm, pos, types):
    """Fix the four degeneracies against reference antennas.

    Amplitude: sum_i ln|g_i| = 0.  Phase and both phase slopes: the gains of
    the first antenna in raster order and of its +x and +y neighbours
    ((0,0), (1,0) and (0,1) on a square grid) become real and positive.  Because
    positions are integers the slope transform is 2 pi periodic, so no phase
    unwrapping is involved.  V_alpha absorbs the compensating transform.
    """
    g = np.array(g, dtype=np.complex128)
    vm = np.array(vm, dtype=np.complex128)
    d = np.asarray(types, dtype=float)
    lam = np.exp(np.mean(np.log(np.abs(g))))
    g = g / lam
    vm = vm * lam ** 2
    a0, ax, ay, rel = _ref_antennas(pos)
    th0 = np.angle(g[a0])
    thx = np.angle(g[ax] * np.conj(g[a0]))
    thy = np.angle(g[ay] * np.conj(g[a0]))
    g = g * np.exp(-1j * (th0 + thx * rel[:, 0] + thy * rel[:, 1]))
    vm = vm * np.exp(1j * (thx * d[:, 0] + thy * d[:, 1]))
    return g, vm


def fix_match(g, vm, g_ref, pos, types):
    """Fix the degeneracies by matching reference gains (Sec. 3 procedure).

    Amplitude: mean ln|g| = mean ln|g_ref|.  Phase: least-squares plane
    c + k_x x + k_y y fitted to the wrapped arg(g_i conj(g_ref_i)) and
    removed.  Only meaningful when g is already close to g_ref.
    """
    g = np.array(g, dtype=np.complex128)
    vm = np.array(vm, dtype=np.complex128)
    d = np.asarray(types, dtype=float)
    r = np.asarray(pos, dtype=float)
    lam = np.exp(np.mean(np.log(np.abs(g))) - np.mean(np.log(np.abs(g_ref))))
    g = g / lam
    vm = vm * lam ** 2
    dphi = np.angle(g * np.conj(g_ref))
    a = np.stack([np.ones(len(g)), r[:, 0], r[:, 1]], axis=1)
    c = np.linalg.lstsq(a, dphi, rcond=None)[0]
    g = g * np.exp(-1j * (a @ c))
    vm = vm * np.exp(1j * (c[1] * d[:, 0] + c[2] * d[:, 1]))
    return g, vm


# ----------------------------------------------------------------------- driver

def calibrate(vred, pos, types, pairs, tix, init: Optional[Tuple[np.ndarray, np.ndarray]] = None,
              solver: str = "lincal", fix: str = "refant", g_ref=None, tol: float = 1e-10):
    """Full reduced redundant calibration of one unit.

    Returns dict(g, vm, chisq, dof, niter, converged) with the degeneracies
    fixed by `fix` ("refant" or "match").
    """
    if init is None:
        g0, v0 = firstcal(vred, pos, types, pairs, tix)
    else:
        g0, v0 = init
    if solver == "lincal":
        g, vm, it, ok = lincal(vred, pos, types, pairs, tix, g0, v0, tol=tol)
    else:
        g, vm, it, ok = omnical(vred, pairs, tix, g0, v0, tol=tol)
    if fix == "refant":
        g, vm = fix_refant(g, vm, pos, types)
    else:
        g, vm = fix_match(g, vm, g_ref, pos, types)
    return dict(g=g, vm=vm, chisq=chisq(vred, g, vm, pairs, tix),
                dof=dof(len(pairs), len(pos), len(types)), niter=it, converged=ok)
