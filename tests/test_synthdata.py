"""The input generator: determinism, the sky's power law, SNR and gains."""
import numpy as np

from synthdata import WORKLOADS, sky_power, unit_gains, unit_voltages, workload_voltages


def test_deterministic_and_independent():
    g = unit_gains(1, 0, 4, 3, True)
    a = unit_voltages(1, 0, 2, 4, 8, 64, 10.0, g[2])
    b = unit_voltages(1, 0, 2, 4, 8, 64, 10.0, g[2])
    c = unit_voltages(1, 0, 1, 4, 8, 64, 10.0, g[2])
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    assert np.array_equal(unit_voltages(1, 0, 2, 4, 8, 64, 10.0, g[2], t_slice=slice(3, 9)), a[3:9])


def test_sky_power_law():
    p = sky_power(16)
    assert p[0, 0] == 0.0 and abs(p.sum() - 1.0) < 1e-15
    # P_k |k|^2 is constant away from k = 0
    assert abs(p[0, 1] * 1 - p[3, 4] * 25) < 1e-15
    assert abs(p[0, 15] - p[0, 1]) < 1e-15          # centred frequency: index 15 is k = -1


def test_gain_statistics_and_drift():
    g = unit_gains(1, 0, 32, 8, True)
    amp = np.abs(g[0])
    assert abs(amp.mean() - 1) < 0.01 and abs(amp.std() - 0.05) < 0.01
    slope = np.angle(g[1] * np.conj(g[0]))
    assert np.all(np.abs(slope) <= 0.1 + 1e-12)
    assert np.allclose(np.abs(g[5]), amp)
    g0 = unit_gains(0, 0, 8, 2, False)
    assert np.array_equal(g0[0], g0[1])


def test_noise_level_and_signal_power():
    n, m, t = 8, 16, 4096
    g = np.ones(n * n)
    sig = unit_voltages(0, 0, 0, n, m, t, 10.0, g, noiseless=True)
    tot = unit_voltages(0, 0, 0, n, m, t, 10.0, g)
    assert abs(np.mean(np.abs(sig) ** 2) - 1.0) < 0.02
    assert abs(np.mean(np.abs(tot - sig) ** 2) - 0.01) < 0.0005


def test_workload_table_shapes():
    w = WORKLOADS[1]
    v, g = workload_voltages(w, 0, chans=[0, 5])
    assert v.shape == (2, 1024, 256) and v.dtype == np.complex64 and g.shape == (2, 256)
    assert [w.pad(n) for n in WORKLOADS[3].grids] == [32, 64, 64, 128]
