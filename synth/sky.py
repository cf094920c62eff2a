"""Seeded synthetic sky-image streams with dispersed point-source transients.

This module only *generates inputs*.  It holds none of the detection
method's arithmetic (no filtering, thresholding, statistics or flux
measurement) so that both the oracle and the device path can read the same
bytes without sharing any of the method's code.

What is simulated (stand-ins for the instrument data the paper uses):

* one image cube per 1 s time step, ``B`` subbands x ``H`` x ``W`` pixels,
  float32, band-major and row-major (Sec. 2.1: the input at time t is a
  B x D x D cube);
* i.i.d. N(0, 1) noise, drawn in float64 and rounded to float32, from a
  Philox generator keyed by ``(seed, cfg, stream, t, band)`` so any frame can
  be regenerated alone;
* optionally a circular sky mask (pixels outside are exactly 0.0; sources
  are placed uniformly in a circle of diameter D as in App. D) and a smooth
  large-scale background standing in for the extended-emission map of
  App. D, which is not available;
* point sources with a circular Gaussian PSF (FWHM 3 px), point-sampled at
  pixel centres, peak value equal to the amplitude;
* a boxcar pulse in time that is delayed per band by the cold-plasma
  dispersion law t_nu = t0 + C_DM * DM * (nu^-2 - nu_max^-2)  (Sec. 3.2),
  integrated over each 1 s frame;
* optional RFI: bright full-row/column stripes or whole-band x5 noise
  (the two corruption modes of App. A).

Pixel (i, j) has its centre at coordinates (i, j) for the PSF; the sky mask
keeps pixel (i, j) iff (i + 1/2 - H/2)^2 + (j + 1/2 - W/2)^2 <= (min(H,W)/2)^2.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Dispersion constant in s * MHz^2 * pc^-1 * cm^3.  The paper quotes
# 4148.806 (Sec. 3.2, with a unit typo); the streams here use 4.15e3.
C_DM = 4.15e3
FWHM_PX = 3.0
SIGMA_PSF = FWHM_PX / (2.0 * math.sqrt(2.0 * math.log(2.0)))
PSF_HALF = int(math.ceil(4.0 * SIGMA_PSF))  # stamp half-width, px

BASE_SEED = 2103_15418


@dataclasses.dataclass
class Source:
    row: float
    col: float
    amp: float
    dm: float
    width: float     # boxcar length in time steps
    t0: float        # arrival time at the top band, s (= time steps)


@dataclasses.dataclass
class StreamSpec:
    """Shape and content recipe of one synthetic stream."""
    name: str
    B: int
    H: int
    W: int
    T: int
    freqs_mhz: np.ndarray
    n_sources: int
    amp: tuple = (8.0, 8.0)          # U(lo, hi); equal => fixed
    dm: tuple = (0.0, 200.0)
    width_choices: tuple = (2,)      # drawn uniformly from these
    t0: tuple = (0.0, 10.0)
    integer_centres: bool = True
    place_box: Optional[tuple] = None   # (lo, hi) for row/col when no mask
    mask: bool = False
    mask_shrink: int = 0             # sources kept this far inside the mask
    min_sep: float = 16.0
    gradient: bool = False
    rfi_p: float = 0.0
    rfi_from_t: int = 8
    seed: int = BASE_SEED
    cfg: int = 0
    stream: int = 0


def two_group_freqs(B: int = 16) -> np.ndarray:
    """Two contiguous groups of 8 subbands with a gap, 58-72 MHz.

    Group one 58 + 0.75 i, group two 66.75 + 0.75 i (i = 0..7).  An 8-band
    stream takes the even-indexed subset.
    """
    f = np.concatenate([58.0 + 0.75 * np.arange(8), 66.75 + 0.75 * np.arange(8)])
    if B == 16:
        return f
    if B == 8:
        return f[::2].copy()
    raise ValueError("two_group_freqs supports B = 16 or 8")


def spec_tiny(seed: Optional[int] = None) -> StreamSpec:
    """4 subbands x 16 steps of 256^2, N(0,1) noise, 5 sources at 8 sigma."""
    return StreamSpec(
        name="tiny", B=4, H=256, W=256, T=16,
        freqs_mhz=np.linspace(60.0, 70.0, 4), n_sources=5,
        amp=(8.0, 8.0), dm=(0.0, 200.0), width_choices=(2,), t0=(0.0, 10.0),
        integer_centres=True, place_box=(24, 232), mask=False,
        seed=BASE_SEED + 1 if seed is None else seed, cfg=1)


def spec_instrument(seed: Optional[int] = None, T: int = 60, H: int = 1024) -> StreamSpec:
    """16 subbands (two groups of 8) x 60 steps of 1024^2 in a circular mask."""
    return StreamSpec(
        name="instrument", B=16, H=H, W=H, T=T,
        freqs_mhz=two_group_freqs(16), n_sources=50,
        amp=(5.0, 20.0), dm=(0.0, 500.0), width_choices=(1, 2, 3, 4),
        t0=(0.0, 50.0), integer_centres=False, mask=True, mask_shrink=48,
        gradient=True, seed=BASE_SEED + 2 if seed is None else seed, cfg=2)


def spec_streaming(seed: Optional[int] = None, T: int = 300, H: int = 2048) -> StreamSpec:
    """16 subbands x 300 steps of 2048^2, 200 sources, 5% RFI (band, step)."""
    return StreamSpec(
        name="streaming", B=16, H=H, W=H, T=T,
        freqs_mhz=two_group_freqs(16), n_sources=200,
        amp=(5.0, 20.0), dm=(0.0, 500.0), width_choices=(1, 2, 3, 4),
        t0=(0.0, 250.0), integer_centres=False, mask=True, mask_shrink=48,
        gradient=True, rfi_p=0.05, seed=BASE_SEED + 3 if seed is None else seed, cfg=3)


def spec_serving_streams(seed: Optional[int] = None, T: int = 600) -> List[StreamSpec]:
    """Eight streams of uneven shape: 2x512^2, 2x1024^2, 2x2048^2 (16 bands)
    and 2x1536^2 with 8 bands; 20 sources each."""
    base = BASE_SEED + 5 if seed is None else seed
    shapes = [(16, 512), (16, 512), (16, 1024), (16, 1024),
              (16, 2048), (16, 2048), (8, 1536), (8, 1536)]
    out = []
    for k, (b, d) in enumerate(shapes):
        out.append(StreamSpec(
            name=f"serve{k}", B=b, H=d, W=d, T=T, freqs_mhz=two_group_freqs(b),
            n_sources=20, amp=(5.0, 20.0), dm=(0.0, 500.0),
            width_choices=(1, 2, 3, 4), t0=(0.0, max(1.0, T - 40.0)),
            integer_centres=False, mask=True, mask_shrink=48, gradient=True,
            seed=base, cfg=5, stream=k))
    return out


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(k) for k in key])))


def sky_mask(H: int, W: int) -> np.ndarray:
    """Circular sky mask of diameter min(H, W), uint8 {0,1}."""
    r = min(H, W) / 2.0
    i = np.arange(H)[:, None] + 0.5 - H / 2.0
    j = np.arange(W)[None, :] + 0.5 - W / 2.0
    return ((i * i + j * j) <= r * r).astype(np.uint8)


def arrival_times(src: Source, freqs_mhz: Sequence[float]) -> np.ndarray:
    """Per-band pulse start: t0 + C_DM * DM * (nu^-2 - nu_max^-2)."""
    f = np.asarray(freqs_mhz, dtype=np.float64)
    return src.t0 + C_DM * src.dm * (f ** -2 - f.max() ** -2)


def boxcar_overlap(t_start: float, width: float, tau: int) -> float:
    """Length of [tau, tau+1) intersected with [t_start, t_start + width)."""
    lo = max(float(tau), t_start)
    hi = min(float(tau) + 1.0, t_start + width)
    return max(0.0, hi - lo)


class Stream:
    """A deterministic synthetic stream; ``frame(t)`` regenerates step t."""

    def __init__(self, spec: StreamSpec):
        self.spec = spec
        s = spec
        self.freqs = np.asarray(s.freqs_mhz, dtype=np.float64)
        self.mask = sky_mask(s.H, s.W) if s.mask else None
        self.sources = self._draw_sources()
        self.arrivals = np.array([arrival_times(src, self.freqs) for src in self.sources]
                                 ).reshape(len(self.sources), s.B)
        self._bg = self._background() if s.gradient else None
        self.rfi = self._draw_rfi()

    # -- catalogue -----------------------------------------------------------------
    def _draw_sources(self) -> List[Source]:
        s = self.spec
        g = _rng(s.seed, s.cfg, s.stream, 1_000_001)
        out: List[Source] = []
        tries = 0
        while len(out) < s.n_sources:
            tries += 1
            if tries > 100000:
                raise RuntimeError("could not place sources")
            if s.mask:
                rad = min(s.H, s.W) / 2.0 - s.mask_shrink
                rr = rad * math.sqrt(g.uniform())
                th = g.uniform(0.0, 2.0 * math.pi)
                row = s.H / 2.0 - 0.5 + rr * math.sin(th)
                col = s.W / 2.0 - 0.5 + rr * math.cos(th)
            else:
                lo, hi = s.place_box if s.place_box else (0, min(s.H, s.W))
                row = g.uniform(lo, hi)
                col = g.uniform(lo, hi)
            if s.integer_centres:
                row, col = float(int(row)), float(int(col))
            if any((row - o.row) ** 2 + (col - o.col) ** 2 < s.min_sep ** 2 for o in out):
                continue
            amp = s.amp[0] if s.amp[0] == s.amp[1] else g.uniform(*s.amp)
            dm = g.uniform(*s.dm)
            width = float(s.width_choices[int(g.integers(len(s.width_choices)))])
            t0 = g.uniform(*s.t0)
            out.append(Source(row, col, float(amp), float(dm), width, float(t0)))
        return out

    def _background(self) -> np.ndarray:
        s = self.spec
        g = _rng(s.seed, s.cfg, s.stream, 1_000_002)
        D = min(s.H, s.W)
        p0 = (g.uniform(0.25, 0.75) * s.H, g.uniform(0.25, 0.75) * s.W)
        yh = (np.arange(s.H)[:, None] + 0.5) / s.H - 0.5
        xh = (np.arange(s.W)[None, :] + 0.5) / s.W - 0.5
        ii = np.arange(s.H)[:, None] + 0.5
        jj = np.arange(s.W)[None, :] + 0.5
        d2 = (ii - p0[0]) ** 2 + (jj - p0[1]) ** 2
        return 1.5 * (xh + 0.5 * yh) + 1.0 * np.exp(-d2 / (2.0 * (D / 4.0) ** 2))

    def _draw_rfi(self) -> dict:
        """{(t, band): ("stripe", [(axis, index, amp)...]) | ("noise5", None)}"""
        s = self.spec
        out = {}
        if s.rfi_p <= 0:
            return out
        for t in range(s.rfi_from_t, s.T):
            for b in range(s.B):
                g = _rng(s.seed, s.cfg, s.stream, t, b, 2_000_003)
                if g.uniform() >= s.rfi_p:
                    continue
                if g.uniform() < 0.5:
                    n = int(g.integers(1, 5))
                    lines = []
                    for _ in range(n):
                        axis = int(g.integers(2))
                        idx = int(g.integers(min(s.H, s.W) // 4, 3 * min(s.H, s.W) // 4))
                        lines.append((axis, idx, float(g.uniform(20.0, 100.0))))
                    out[(t, b)] = ("stripe", lines)
                else:
                    out[(t, b)] = ("noise5", None)
        return out

    # -- per-step content ------------------------------------------------------------
    def amplitude(self, k: int, t: int, b: int) -> float:
        src = self.sources[k]
        return src.amp * boxcar_overlap(self.arrivals[k, b], src.width, t)

    def psf_stamp(self, k: int):
        """(rows, cols, values) of the unit-peak PSF of source k, clipped to the image."""
        src = self.sources[k]
        s = self.spec
        r0, c0 = int(round(src.row)), int(round(src.col))
        rs = np.arange(max(0, r0 - PSF_HALF), min(s.H, r0 + PSF_HALF + 1))
        cs = np.arange(max(0, c0 - PSF_HALF), min(s.W, c0 + PSF_HALF + 1))
        d2 = (rs[:, None] - src.row) ** 2 + (cs[None, :] - src.col) ** 2
        return rs, cs, np.exp(-d2 / (2.0 * SIGMA_PSF ** 2))

    def band_image(self, t: int, b: int, noise: bool = True) -> np.ndarray:
        s = self.spec
        rfi = self.rfi.get((t, b))
        if noise:
            img = _rng(s.seed, s.cfg, s.stream, t, b).standard_normal((s.H, s.W))
            if rfi is not None and rfi[0] == "noise5":
                img *= 5.0
        else:
            img = np.zeros((s.H, s.W))
        if self._bg is not None:
            img += self._bg
        for k in range(len(self.sources)):
            a = self.amplitude(k, t, b)
            if a > 0.0:
                rs, cs, v = self.psf_stamp(k)
                img[rs[0]:rs[-1] + 1, cs[0]:cs[-1] + 1] += a * v
        if rfi is not None and rfi[0] == "stripe":
            for axis, idx, amp in rfi[1]:
                if axis == 0:
                    img[idx, :] += amp
                else:
                    img[:, idx] += amp
        if self.mask is not None:
            img *= self.mask
        return img.astype(np.float32)

    def frame(self, t: int, noise: bool = True) -> np.ndarray:
        """float32 [B][H][W] cube for step t (contiguous)."""
        s = self.spec
        out = np.empty((s.B, s.H, s.W), dtype=np.float32)
        for b in range(s.B):
            out[b] = self.band_image(t, b, noise)
        return out

    def rfi_mask(self, t: int) -> int:
        """Bitmask of bands carrying injected RFI at step t."""
        m = 0
        for b in range(self.spec.B):
            if (t, b) in self.rfi:
                m |= 1 << b
        return m
