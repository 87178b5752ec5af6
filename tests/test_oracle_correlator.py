"""Pins for oracle.correlator: brute force, the convolution theorem behind the
FFT-correlator, a closed-form single-mode sky, Parseval and the exact
integer X-engine."""
import numpy as np
import pytest

from oracle import correlator as C
from oracle import geometry as G
from synthdata import pack_ci4, unpack_ci4, quantise_ci4


def _rand_volt(rng, t, n):
    return rng.standard_normal((t, n)) + 1j * rng.standard_normal((t, n))


def test_fx_bruteforce():
    rng = np.random.default_rng(1)
    v = _rand_volt(rng, 5, 6)
    ref = np.zeros((6, 6), dtype=complex)
    for i in range(6):
        for j in range(6):
            s = 0j
            for t in range(5):
                s += v[t, i] * np.conj(v[t, j])
            ref[i, j] = s / 5
    assert np.allclose(C.fx_correlate(v), ref, rtol=0, atol=1e-14)
    vf = C.fx_correlate(v)
    assert np.allclose(vf, vf.conj().T, atol=1e-15)       # V_ji = conj(V_ij)


@pytest.mark.parametrize("n", [2, 3])
def test_redundant_average_bruteforce(n):
    rng = np.random.default_rng(n)
    v = _rand_volt(rng, 4, n * n)
    g = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    pos = G.square_positions(n)
    types, _ = G.square_types(n)
    out = C.redundant_average(C.fx_correlate(v), g, pos, types)
    for t, (dx, dy) in enumerate(types):
        acc, cnt = 0j, 0
        for i in range(n * n):
            for j in range(n * n):
                if pos[i, 0] - pos[j, 0] == dx and pos[i, 1] - pos[j, 1] == dy:
                    acc += np.mean(v[:, i] * np.conj(v[:, j])) / (g[i] * np.conj(g[j]))
                    cnt += 1
        assert abs(out[t] - acc / cnt) < 1e-13


def _fft_route(w, n, m):
    """Convolution theorem (Sec. 1): zero-padded spatial FFT, |.|^2, sum, inverse FFT."""
    t = w.shape[0]
    grid = np.zeros((t, m, m), dtype=complex)
    grid[:, :n, :n] = w.reshape(t, n, n)              # [t, y, x]
    e = np.fft.fft2(grid, axes=(1, 2))
    p = np.sum(np.abs(e) ** 2, axis=0)
    return np.fft.ifft2(p)                            # C[dy mod m, dx mod m]


@pytest.mark.parametrize("n,m", [(3, 6), (4, 8), (5, 16), (8, 16)])
def test_fft_correlator_identity(n, m):
    rng = np.random.default_rng(10 + n)
    t = 7
    v = _rand_volt(rng, t, n * n)
    g = (1 + 0.1 * rng.standard_normal(n * n)) * np.exp(1j * rng.uniform(-np.pi, np.pi, n * n))
    w = v / g[None, :]
    c = _fft_route(w, n, m)
    pos = G.square_positions(n)
    lags = C.canonical_lags(n)
    ref = C.redundant_average(C.fx_correlate(v), g, pos, lags)
    for k, (dx, dy) in enumerate(lags):
        nd = (n - abs(dx)) * (n - abs(dy))
        assert abs(c[dy % m, dx % m] / (nd * t) - ref[k]) < 1e-12
    assert abs(c[0, 0].real / (n * n * t) - C.calibrated_auto(C.fx_correlate(v), g)) < 1e-12


def test_single_mode_closed_form():
    # One sky mode k0, no noise, unit gains: V(d) = <|s|^2> exp(-2 pi i k0.d / M).
    n, m, t = 6, 12, 9
    rng = np.random.default_rng(3)
    s = rng.standard_normal(t) + 1j * rng.standard_normal(t)
    k0 = np.array([2, 5])
    pos = G.square_positions(n)
    v = s[:, None] * np.exp(-2j * np.pi * (pos @ k0) / m)[None, :]
    lags = C.canonical_lags(n)
    out = C.redundant_average(C.fx_correlate(v), np.ones(n * n), pos, lags)
    p = np.mean(np.abs(s) ** 2)
    for k, d in enumerate(lags):
        assert abs(out[k] - p * np.exp(-2j * np.pi * (k0 @ np.array(d)) / m)) < 1e-13


def test_parseval_zero_lag():
    rng = np.random.default_rng(4)
    v = _rand_volt(rng, 11, 9)
    g = 1 + 0.2 * rng.standard_normal(9) + 0.2j * rng.standard_normal(9)
    w = v / g
    assert abs(C.calibrated_auto(C.fx_correlate(v), g) - np.sum(np.abs(w) ** 2) / w.size) < 1e-13


def test_canonical_lags():
    for n in [2, 5, 9]:
        lags = C.canonical_lags(n)
        assert len(lags) == 2 * n * (n - 1)
        assert sorted(lags) == sorted(G.square_types(n)[0])
        assert all(G.is_canonical(dx, dy) for dx, dy in lags)


def test_xengine_int_bruteforce():
    rng = np.random.default_rng(5)
    t, n = 6, 3
    re = rng.integers(-7, 8, (t, n * n))
    im = rng.integers(-7, 8, (t, n * n))
    pos = G.square_positions(n)
    pairs, _ = G.group_pairs(pos, G.square_types(n)[0])
    out = C.xengine_int(re, im, pairs)
    for p, (i, j) in enumerate(pairs):
        sr = si = 0
        for k in range(t):
            q1 = complex(int(re[k, i]), int(im[k, i]))
            q2 = complex(int(re[k, j]), int(im[k, j]))
            z = q1 * q2.conjugate()
            sr += int(z.real)
            si += int(z.imag)
        assert out[p, 0] == sr and out[p, 1] == si
    # same products as the float correlator on the same small integers
    vf = C.fx_correlate(re + 1j * im) * t
    assert np.array_equal(out[:, 0], np.rint(vf[pairs[:, 0], pairs[:, 1]].real).astype(np.int64))
    assert np.array_equal(out[:, 1], np.rint(vf[pairs[:, 0], pairs[:, 1]].imag).astype(np.int64))


def test_xengine_float_gathers_pairs():
    rng = np.random.default_rng(6)
    v = _rand_volt(rng, 8, 16)
    pos = G.square_positions(4)
    pairs, _ = G.group_pairs(pos, [(1, 0), (0, 1), (-1, 1)])
    out = C.xengine(C.fx_correlate(v), pairs)
    for p, (i, j) in enumerate(pairs):
        assert abs(out[p] - np.mean(v[:, i] * np.conj(v[:, j]))) < 1e-14


def test_ci4_pack_roundtrip():
    vals = np.arange(-7, 8)
    re, im = np.meshgrid(vals, vals)
    re, im = re.ravel().astype(np.int8), im.ravel().astype(np.int8)
    b = pack_ci4(re, im)
    r2, i2 = unpack_ci4(b)
    assert np.array_equal(r2, re) and np.array_equal(i2, im)
    assert pack_ci4(np.array([-1], np.int8), np.array([2], np.int8))[0] == 0xF2


def test_ci4_quantise_scale():
    rng = np.random.default_rng(7)
    v = 3.0 * (rng.standard_normal(20000) + 1j * rng.standard_normal(20000))
    re, im = quantise_ci4(v)
    assert re.min() >= -7 and re.max() <= 7 and im.min() >= -7 and im.max() <= 7
    rms = np.sqrt(np.mean(re.astype(float) ** 2 + im.astype(float) ** 2) / 2)
    assert abs(rms - 2.5) < 0.05


def test_redundant_average_on_a_masked_lattice():
    # a lag that no pair of the hexagon realises is reported as zero; the
    # others are the brute-force group means
    n, _, pos = G.hex_grid(3)
    rng = np.random.default_rng(11)
    v = rng.standard_normal((40, len(pos))) + 1j * rng.standard_normal((40, len(pos)))
    g = np.exp(0.1 * rng.standard_normal(len(pos)) + 1j * rng.uniform(-1, 1, len(pos)))
    vf = C.fx_correlate(v)
    lags = C.canonical_lags(n)
    out = C.redundant_average(vf, g, pos, lags)
    empty = 0
    for t, (dx, dy) in enumerate(lags):
        members = [(i, j) for i in range(len(pos)) for j in range(len(pos))
                   if pos[i, 0] - pos[j, 0] == dx and pos[i, 1] - pos[j, 1] == dy]
        if not members:
            assert out[t] == 0
            empty += 1
        else:
            want = np.mean([vf[i, j] / (g[i] * np.conj(g[j])) for i, j in members])
            assert abs(out[t] - want) <= 1e-12 * abs(want)
    assert empty > 0
