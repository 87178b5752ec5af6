"""The same synthetic instrument model as `generate.py`, drawn on the GPU.

For the multi-gigabyte workloads (32x32 and larger grids, hundreds of
channels) host generation would dominate the run, so the voltages are drawn
with torch on the device, following the recipe of `generate.py`:

* sky s_k(t) ~ CN(0, P_k) on the M x M mode grid (P_k as `sky_power`);
* u(x, t) = sum_k s_k(t) exp(-2 pi i k.x / M) at the n x n antenna points;
* gains from `unit_gains` (identical values to the host generator);
* noise n ~ CN(0, 1/SNR^2); v = g u + n;
* 4-bit: per unit, scale to rms 2.5 per real component, round half to
  even, clip to [-7, 7], pack (re << 4) | (im & 0xF).

The random numbers come from torch's device generator seeded from
SeedSequence([20050306, workload, array, channel]), so the values differ
from the host generator's (same distribution, not the same bytes); a test
or check that compares with the oracle copies the sampled units' bytes back
to the host and feeds the oracle exactly those.  Like `generate.py`, this
module contains none of the method's arithmetic.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import torch

from .generate import ROOT_SEED, Workload, sky_power, unit_gains


def _seed(wid: int, array: int, chan: int) -> int:
    ss = np.random.SeedSequence([ROOT_SEED, wid, array, chan])
    return int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1))


def device_voltages(w: Workload, array: int, device, block: int = 256) -> Tuple[torch.Tensor, np.ndarray]:
    """Voltages [C, T, N] (complex64, or packed uint8 for 4-bit workloads)
    and the gains [C, N] (complex128, host) of one array of workload w."""
    n = w.grids[array]
    m = w.pad(n)
    nant = n * n
    C, T = w.n_chan, w.n_time
    gains = unit_gains(w.wid, array, n, C, w.drift)
    amp = torch.from_numpy(np.sqrt(sky_power(m) / 2.0).astype(np.float32)).to(device)
    sig = float(np.sqrt(0.5) / w.snr)
    out = torch.empty((C, T, nant), dtype=torch.uint8 if w.ci4 else torch.complex64, device=device)
    gen = torch.Generator(device=device)
    for c in range(C):
        gen.manual_seed(_seed(w.wid, array, c))
        g = torch.from_numpy(gains[c].astype(np.complex64)).to(device)
        v = torch.empty((T, nant), dtype=torch.complex64, device=device)
        for t0 in range(0, T, block):
            nb = min(block, T - t0)
            re = torch.randn((nb, m, m), generator=gen, device=device) * amp
            im = torch.randn((nb, m, m), generator=gen, device=device) * amp
            u = torch.fft.fft2(torch.complex(re, im))[:, :n, :n].reshape(nb, nant)
            nz = torch.complex(torch.randn((nb, nant), generator=gen, device=device),
                               torch.randn((nb, nant), generator=gen, device=device)) * sig
            v[t0:t0 + nb] = g[None, :] * u + nz
        if w.ci4:
            rms = torch.sqrt(torch.mean(v.real.double() ** 2 + v.imag.double() ** 2) / 2.0)
            s = (2.5 / rms).float()
            qre = torch.clamp(torch.round(v.real * s), -7, 7).to(torch.int16)
            qim = torch.clamp(torch.round(v.imag * s), -7, 7).to(torch.int16)
            out[c] = (((qre << 4) & 0xF0) | (qim & 0x0F)).to(torch.uint8)
        else:
            out[c] = v
    return out, gains
