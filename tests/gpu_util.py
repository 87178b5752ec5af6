"""Shared helpers of the GPU parity tests: seeded inputs, oracle references
and the tolerances they are held to."""
import numpy as np

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import redcal as OR
from synthdata import WORKLOADS, Workload, pack_ci4, quantise_ci4, unit_gains, unit_voltages

# V^unique: relative L2 over the lag vector of a unit, same gains on both
# sides (the correlator's FP32 error alone).
TOL_VUNIQUE = 1e-5
# Gains after the same degeneracy convention, both solvers fed the same
# V^reduced: the oracle's own (FP64 from the voltages, or exact integer sums
# for 4-bit data), rounded to complex64 for the GPU's input and promoted back
# for the oracle's (the rounding is the test's, so both see identical values).
TOL_GAINS = 1e-6
# Gains of the whole float path (GPU X-engine in FP32, then the solve)
# against the oracle's whole chain in FP64.  The X-engine's rounding
# (TOL_XENG below bounds it relative to the mean power) reaches the gains
# through the solve's sensitivity, which grows with the grid and falls with
# SNR: measured 2e-7 .. 6e-7 at 16x16 (SNR 10) and 1.4e-5 at 32x32 (SNR 5).
# 1e-4 bounds it with margin; the solver alone is held to TOL_GAINS.
TOL_GAINS_E2E = 1e-4
# omnical's FP32 iteration (no FP64 refinement) stopped at a relative change
# Delta = 1e-7: the distance left to the minimum is about Delta / (eta (1 -
# rho)) with eta = 0.3 the damping and rho the contraction of the slowest
# (long-wavelength phase) mode, which approaches 1 as the grid grows:
# measured 5.7e-6 at 8x8 and 2.3e-5 at 16x16 (chi^2 within 3e-8 of the
# minimum's).  The bar is 1e-4.
TOL_OMNICAL = 1e-4
# FP32 X-engine: |dV_b| relative to the unit's mean voltage power.  T
# products of |v|^2 ~ 1 summed in FP32 in runs of at most a few hundred
# samples: a random-walk rounding error of ~sqrt(T) * 6e-8 < 4e-6 for
# T <= 4096; 2e-5 leaves margin for the worst case.
TOL_XENG = 2e-5


def make_units(n, n_units, n_time, wid=90, snr=10.0, drift=False, array=0):
    """complex64 voltages [U, T, N] and complex128 gains [U, N] (seeded)."""
    m = 16
    while m < 2 * n:
        m *= 2
    g = unit_gains(wid, array, n, n_units, drift)
    v = np.empty((n_units, n_time, n * n), dtype=np.complex64)
    for c in range(n_units):
        v[c] = unit_voltages(wid, array, c, n, m, n_time, snr, g[c]).astype(np.complex64)
    return v, g


def make_ci4_units(n, n_units, n_time, wid=91):
    v, g = make_units(n, n_units, n_time, wid=wid)
    out = np.empty(v.shape, dtype=np.uint8)
    re_all = np.empty(v.shape, dtype=np.int8)
    im_all = np.empty(v.shape, dtype=np.int8)
    for c in range(n_units):
        re, im = quantise_ci4(v[c].astype(np.complex128))
        re_all[c], im_all[c] = re, im
        out[c] = pack_ci4(re, im)
    return out, re_all, im_all, g


def oracle_vunique(v_unit, gains, n):
    pos = OG.square_positions(n)
    vf = OC.fx_correlate(v_unit.astype(np.complex128))
    lags = OC.canonical_lags(n)
    return OC.redundant_average(vf, gains, pos, lags), OC.calibrated_auto(vf, gains)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def pairs_of(n, types):
    return OG.group_pairs(OG.square_positions(n), types)


def oracle_solve(vred64, n, types, fix="refant", g_ref=None, init=None):
    pos = OG.square_positions(n)
    pairs, tix = OG.group_pairs(pos, types)
    return OR.calibrate(vred64, pos, types, pairs, tix, fix=fix, g_ref=g_ref, init=init)


def oracle_vred(v_unit, pairs):
    """The oracle's V^reduced of one float unit (FP64 X-engine of the FX matrix)."""
    return OC.xengine(OC.fx_correlate(v_unit.astype(np.complex128)), pairs)


def as_c64(x):
    """complex64 rounding of an oracle value, and that rounding promoted back."""
    x32 = np.asarray(x).astype(np.complex64)
    return x32, x32.astype(np.complex128)


def ci4_sums_int32(sums_i64):
    """[P, 2] exact int64 sums as the int32 pairs a 4-bit plan's solve reads."""
    s = np.asarray(sums_i64)
    assert np.all(np.abs(s) < 2 ** 31)
    return s.astype(np.int32)


def gain_err(g_gpu, g_ref):
    g = np.asarray(g_gpu).astype(np.complex128)
    return float(np.max(np.abs(g - g_ref) / np.abs(g_ref)))
