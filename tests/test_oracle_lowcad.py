"""Pins of the low-cadence oracle (Sec. 4): the round-robin schedule covers
every redundant group once and whole, within the p N log N budget of
eq. lowcadcal_inttime; the populated matrix is the FX correlator over each
cycle's samples (brute force); one cycle is the full FX matrix; and the
predicted gain variance of the populated matrix follows eq. gainvar_lowcadcal
(proportional to 1 / (p log N) at a fixed calibration interval)."""
import math

import numpy as np
import pytest

from oracle import correlator as C
from oracle import geometry as G
from oracle import lowcad as LC
from oracle import stats as OS


@pytest.mark.parametrize("n,p", [(4, 1.0), (6, 1.0), (8, 0.5), (12, 1.0), (16, 2.0)])
def test_schedule_whole_groups_within_budget(n, p):
    lags = C.canonical_lags(n)
    N = n * n
    b = LC.budget(N, p)
    cyc = LC.schedule(n, p)
    assert cyc[0][0] == 0 and cyc[-1][1] == len(lags)
    sizes = [(n - abs(dx)) * (n - dy) for dx, dy in lags]
    for k, (t0, t1) in enumerate(cyc):
        assert t1 > t0
        if k:
            assert t0 == cyc[k - 1][1]                      # contiguous, each group once
        cnt = sum(sizes[t0:t1])
        assert cnt <= b or t1 == t0 + 1                     # within budget (a lone group may not be)
        if k + 1 < len(cyc):
            assert cnt + sizes[t1] > b                      # a cycle takes groups while they fit
    # eq. lowcadcal_inttime: t_int / t_cal = 1 / N_cycle ~ p N log N / (N^2 / 2)
    total = N * (N - 1) / 2
    assert total / b <= len(cyc) <= total / (b - max(sizes)) + 1


def test_visibilities_brute_force():
    n, T = 3, 11
    rng = np.random.default_rng(3)
    v = rng.standard_normal((T, n * n)) + 1j * rng.standard_normal((T, n * n))
    cyc = LC.schedule(n, p=0.3)
    assert len(cyc) > 2
    got = LC.visibilities(v, n, cyc)
    lags = C.canonical_lags(n)
    rng_s = LC.sample_ranges(T, len(cyc))
    b = 0
    for t, (dx, dy) in enumerate(lags):
        c = [k for k, (t0, t1) in enumerate(cyc) if t0 <= t < t1][0]
        s0, s1 = rng_s[c]
        for y in range(n):
            for x in range(n):
                jx, jy = x - dx, y - dy
                if not (0 <= jx < n and 0 <= jy < n):
                    continue
                i, j = y * n + x, jy * n + jx
                ref = sum(v[s, i] * np.conj(v[s, j]) for s in range(s0, s1)) / (s1 - s0)
                assert abs(got[b] - ref) < 1e-12
                b += 1
    assert b == len(got)


def test_one_cycle_is_the_full_fx_matrix():
    n, T = 5, 40
    rng = np.random.default_rng(4)
    v = rng.standard_normal((T, n * n)) + 1j * rng.standard_normal((T, n * n))
    cyc = LC.schedule(n, p=100.0)
    assert len(cyc) == 1
    pairs, _ = G.group_pairs(G.square_positions(n), C.canonical_lags(n))
    ref = C.xengine(C.fx_correlate(v), pairs)
    assert np.max(np.abs(LC.visibilities(v, n, cyc) - ref)) < 1e-12


def test_gain_variance_follows_one_over_p_log_n():
    # eq. gainvar_lowcadcal: at a fixed calibration interval each cycle gets
    # t_cal / N_cycle, so the visibility SNR^2 falls by N_cycle and the
    # full-matrix variance (~ SNR^-2 / N, eq. gainvar_redcal) becomes
    # N_cycle / (N SNR^2) ~ 1 / (2 p log N SNR^2)
    p, snr2 = 1.0, 1.0
    s = []
    for n in (8, 10, 12, 14, 16):
        N = n * n
        lags = C.canonical_lags(n)
        pos = G.square_positions(n)
        pairs, tix = G.group_pairs(pos, lags)
        ncyc = len(LC.schedule(n, p))
        var = OS.predicted_gain_variance(pos, pairs, tix, len(lags), snr=math.sqrt(snr2 / ncyc)).mean()
        s.append(var * 2 * p * math.log(N) * snr2)
    s = np.array(s)
    # the product is flat in N (whole-group packing and the finite-N excess
    # of the 1/N law move it by a few per cent)
    assert s.max() / s.min() < 1.15
    assert np.all(np.abs(s - 1.0) < 0.25)
