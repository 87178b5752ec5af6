"""Visibility-level simulation of the paper's Sec. 3 (seeded).

The instrument model at the visibility level: for each selected pair
b = (i, j) of type alpha, V_b = g_i conj(g_j) V_alpha + n_b.  The true
visibilities have one amplitude for every type and uniformly random
phases, drawn afresh for each unit (a unit is one realisation); the gains
are drawn once and shared by every unit; n_b is complex Gaussian with
E|n_b|^2 = |g_i g_j V_alpha|^2 / SNR^2, the same SNR on every visibility.
Nothing here calibrates or correlates.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def simulate_reduced_visibilities(seed: int, pairs: np.ndarray, tix: np.ndarray, n_ant: int, n_types: int,
                                  n_units: int, snr: float, gain_scatter: float = 0.0,
                                  amplitude: float = 1.0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(vred [U, P] complex128, gains [N] complex128, true visibilities [U, K]).

    Gain amplitudes are 1 + gain_scatter * N(0, 1) and gain phases uniform."""
    rng = np.random.default_rng(seed)
    g = (1.0 + gain_scatter * rng.standard_normal(n_ant)) * np.exp(2j * np.pi * rng.random(n_ant))
    vm = amplitude * np.exp(2j * np.pi * rng.random((n_units, n_types)))
    noise = (rng.standard_normal((n_units, len(pairs))) + 1j * rng.standard_normal((n_units, len(pairs)))) / np.sqrt(2.0)
    model = g[pairs[:, 0]] * np.conj(g[pairs[:, 1]]) * vm[:, tix]
    return model + np.abs(model) / snr * noise, g, vm
