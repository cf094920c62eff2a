"""Simulated dynamic spectra for training and evaluating the parameter-
inference network (Sec. 3.2).  Generation only: no arithmetic of the
detection method.

Per sample: a Gaussian pulse profile f(t) = exp(-((t - t_nu) / w)^2) with
width w ~ U(0, 16) steps, arrival t_nu = t0 + C_DM DM (nu^-2 - nu_0^-2)
(nu_0 the top band, C_DM as in synth.sky), DM ~ U(0, 512), amplitude
A ~ U(0, 8) noise units and spectral index alpha ~ U(-4, 4), so that
I(t, nu) = A (nu / nu_0)^alpha f(t); t0 ~ U(0, 64).  The pulse is evaluated
at the integer steps t = 0..63 of each band's row of the 16 x 64 grid
(bands of the two-group layout, 58-72 MHz) and added to N(0, 1) noise.
Targets: (DM, w, A, t0).
"""

from __future__ import annotations

import numpy as np

from .sky import C_DM, two_group_freqs

RANGES = {"dm": (0.0, 512.0), "width": (0.0, 16.0), "amp": (0.0, 8.0), "alpha": (-4.0, 4.0), "t0": (0.0, 64.0)}


def simulate(n: int, seed: int, B: int = 16, T: int = 64, noise: bool = True):
    """(x float32 [n][16][T], theta float32 [n][4] = (DM, w, A, t0), alpha [n])."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 5_000_005])))
    nu = two_group_freqs(B)
    nu0 = nu.max()
    dm = g.uniform(*RANGES["dm"], n)
    w = g.uniform(*RANGES["width"], n)
    A = g.uniform(*RANGES["amp"], n)
    al = g.uniform(*RANGES["alpha"], n)
    t0 = g.uniform(*RANGES["t0"], n)
    delay = C_DM * dm[:, None] * (nu[None, :] ** -2 - nu0 ** -2)          # [n][B]
    t = np.arange(T, dtype=np.float64)
    wz = np.maximum(w, 1e-6)[:, None, None]
    prof = np.exp(-(((t[None, None, :] - (t0[:, None, None] + delay[:, :, None])) / wz) ** 2))
    I = A[:, None, None] * (nu[None, :, None] / nu0) ** al[:, None, None] * prof
    x = g.standard_normal((n, B, T)) if noise else np.zeros((n, B, T))
    x = x + I
    grid = np.zeros((n, 16, T))
    grid[:, [b * (16 // B) for b in range(B)], :] = x
    theta = np.stack([dm, w, A, t0], 1)
    return grid.astype(np.float32), theta.astype(np.float32), al.astype(np.float32)
