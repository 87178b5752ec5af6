"""Seeded synthetic channelised antenna voltages on a regular square grid.

Instrument model (Sec. 3 of the paper simulates redundant arrays with ~10 %
gain scatter at SNR 10; here the simulation is done at voltage level):

    v_i(c, t) = g_i(c) * u(x_i, t) + n_i(t)

* antenna i sits at x_i = (i mod n, i div n) (unit spacing, raster order);
* u(x, t) = sum_k s_k(t) exp(-2 pi i k.x / M) is a random sky drawn on an
  M x M grid of modes k, with s_k ~ CN(0, P_k), P_k proportional to |k_c|^-2
  (k_c the centred integer frequency), P_0 = 0 and sum_k P_k = 1;
* g_i has amplitude 1 + N(0, 0.05) and phase U(-pi, pi); with a drift the
  phase gains tau_i * c, tau_i ~ U(-0.1, 0.1) rad per channel;
* n_i ~ CN(0, 1 / SNR^2), i.e. SNR is an amplitude ratio against the
  unit-power sky.

Streams: the gains of one array come from SeedSequence([20050306, w, a]); the
sky and the noise of one (array, channel) unit come from the two children of
SeedSequence([20050306, w, a, c]) (w = workload id, a = array, c = channel).

The 4-bit workload scales each unit so that the rms of its real components
(real and imaginary parts alike) is 2.5, rounds half to even, clips to
[-7, 7] and packs one complex sample per byte as (re << 4) | (im & 0xF).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

ROOT_SEED = 20050306


@dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload (all arrays share C and T)."""
    wid: int                    # seed component
    name: str
    grids: Sequence[int]        # n of each array (n x n antennas)
    n_chan: int
    n_time: int
    snr: float = 10.0
    drift: bool = False         # per-antenna phase drift across channels
    ci4: bool = False           # 4-bit complex voltages
    note: str = ""

    def pad(self, n: int) -> int:
        """Default padded FFT size: the next power of two >= 2n."""
        m = 1
        while m < 2 * n:
            m *= 2
        return m


WORKLOADS: List[Workload] = [
    Workload(0, "g8_c1_t256", (8,), 1, 256, 10.0,
             note="8x8 grid, 1 channel, 256 samples"),
    Workload(1, "g16_c64_t1024", (16,), 64, 1024, 10.0, drift=True,
             note="16x16 grid, 64 channels, 1024 samples, drifting gains"),
    Workload(2, "g32_c256_t2048", (32,), 256, 2048, 5.0,
             note="32x32 grid, 256 channels, 2048 samples, SNR 5"),
    Workload(3, "g16-24-32-48_c128_t1024", (16, 24, 32, 48), 128, 1024, 10.0,
             note="uneven batch of four grids, 128 channels each"),
    Workload(4, "g64_c1024_t4096_ci4", (64,), 1024, 4096, 10.0, ci4=True,
             note="64x64 grid, 1024 channels, 4096 samples, 4-bit voltages"),
]


def sky_power(m: int) -> np.ndarray:
    """P_k on the m x m mode grid, indexed [ky, kx] (numpy FFT order)."""
    k = np.fft.fftfreq(m, d=1.0 / m)          # centred integer frequencies
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    p = np.zeros((m, m))
    nz = k2 > 0
    p[nz] = 1.0 / k2[nz]
    return p / p.sum()


def unit_gains(wid: int, array: int, n: int, n_chan: int, drift: bool) -> np.ndarray:
    """Complex gains g_i(c), shape [n_chan, n*n], complex128."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, wid, array])))
    nant = n * n
    amp = 1.0 + 0.05 * rng.standard_normal(nant)
    phs = rng.uniform(-np.pi, np.pi, nant)
    tau = rng.uniform(-0.1, 0.1, nant) if drift else np.zeros(nant)
    c = np.arange(n_chan)[:, None]
    return amp[None, :] * np.exp(1j * (phs[None, :] + tau[None, :] * c))


def _streams(wid: int, array: int, chan: int):
    ss = np.random.SeedSequence([ROOT_SEED, wid, array, chan])
    sky_ss, noise_ss = ss.spawn(2)
    return (np.random.Generator(np.random.PCG64(sky_ss)),
            np.random.Generator(np.random.PCG64(noise_ss)))


def unit_voltages(wid: int, array: int, chan: int, n: int, m: int, n_time: int,
                  snr: float, gains: np.ndarray, t_slice: Optional[slice] = None,
                  noiseless: bool = False) -> np.ndarray:
    """Voltages of one (array, channel) unit, shape [T, n*n], complex128.

    ``gains`` is the length-n*n gain vector of this channel.  ``t_slice``
    returns a subset of the samples without changing their values (the
    random streams are drawn for all T samples in fixed-size blocks).
    """
    sky_rng, noise_rng = _streams(wid, array, chan)
    nant = n * n
    p = sky_power(m)
    amp = np.sqrt(p / 2.0)
    sig = np.sqrt(0.5) / snr
    out = np.empty((n_time, nant), dtype=np.complex128)
    blk = 256
    for t0 in range(0, n_time, blk):
        t1 = min(n_time, t0 + blk)
        nb = t1 - t0
        s = (sky_rng.standard_normal((nb, m, m)) + 1j * sky_rng.standard_normal((nb, m, m))) * amp
        # u(x, t) = sum_k s_k(t) exp(-2 pi i k.x / M): the sky seen at the grid points
        u = np.fft.fft2(s, axes=(1, 2))[:, :n, :n].reshape(nb, nant)
        nz = (noise_rng.standard_normal((nb, nant)) + 1j * noise_rng.standard_normal((nb, nant))) * sig
        out[t0:t1] = gains[None, :] * u + (0.0 if noiseless else nz)
    if t_slice is not None:
        out = out[t_slice]
    return out


def quantise_ci4(v: np.ndarray):
    """Scale to rms 2.5 per real component, round half-even, clip to [-7, 7].

    Returns (re, im) as int8 arrays of v's shape.
    """
    rms = np.sqrt(np.mean(v.real ** 2 + v.imag ** 2) / 2.0)
    s = 2.5 / rms
    re = np.clip(np.rint(v.real * s), -7, 7).astype(np.int8)
    im = np.clip(np.rint(v.imag * s), -7, 7).astype(np.int8)
    return re, im


def pack_ci4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """One byte per complex sample: high nibble = re, low nibble = im."""
    return ((re.astype(np.int16) << 4) & 0xF0 | (im.astype(np.int16) & 0x0F)).astype(np.uint8)


def unpack_ci4(b: np.ndarray):
    """Inverse of pack_ci4: (re, im) int8 with sign-extended nibbles."""
    b = b.astype(np.int16)
    re = (b >> 4) & 0xF
    im = b & 0xF
    re = np.where(re >= 8, re - 16, re).astype(np.int8)
    im = np.where(im >= 8, im - 16, im).astype(np.int8)
    return re, im


def workload_voltages(w: Workload, array: int, chans: Optional[Sequence[int]] = None,
                      dtype=np.complex64):
    """Voltages [len(chans), T, N] and gains [len(chans), N] of one array.

    complex64 for float workloads; for the 4-bit workload the packed uint8
    bytes [len(chans), T, N] (gains are still returned as complex128).
    """
    n = w.grids[array]
    m = w.pad(n)
    chans = list(range(w.n_chan)) if chans is None else list(chans)
    g_all = unit_gains(w.wid, array, n, w.n_chan, w.drift)
    nant = n * n
    if w.ci4:
        out = np.empty((len(chans), w.n_time, nant), dtype=np.uint8)
    else:
        out = np.empty((len(chans), w.n_time, nant), dtype=dtype)
    for k, c in enumerate(chans):
        v = unit_voltages(w.wid, array, c, n, m, w.n_time, w.snr, g_all[c])
        if w.ci4:
            re, im = quantise_ci4(v)
            out[k] = pack_ci4(re, im)
        else:
            out[k] = v.astype(dtype)
    return out, g_all[chans]
