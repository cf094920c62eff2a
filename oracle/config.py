"""Parameters of the method (oracle side).

Names follow the paper: ``kappa`` is the detection threshold in units of the
local spread (Sec. 2.1.1), ``s`` the Gaussian width, ``k`` half-widths.
Values the paper leaves open carry the readings stated next to them.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KERNEL_GAUSS = 0
KERNEL_BOX = 1
KERNEL_DISK = 2   # circular uniform kernel (Sec. 2.1.1 names it as the alternative)


@dataclasses.dataclass
class OracleConfig:
    B: int
    H: int
    W: int
    freqs_mhz: Optional[np.ndarray] = None
    sky_mask: Optional[np.ndarray] = None   # uint8 [H][W]; None = every pixel
    kappa: float = 4.5                       # Sec. 3.4 uses 4.5 on real data
    s: float = 8.0                           # Gaussian width (px); paper gives heuristics only
    k_bg: int = 0                            # <= 0: ceil(3 s)
    kernel: int = KERNEL_GAUSS               # Gaussian, square uniform, or circular uniform (Sec. 2.1.1)
    n_iter: int = 1                          # sigma-clip iterations (Sec. 3.1 runs one)
    k_peak: int = 3                          # max-filter half-width (Sec. 2.1.2)
    k_flux: int = 2                          # flux box half-width (size unstated)
    r_dup: float = 3.0                       # cross-band duplicate radius, px
    r_assoc: float = 3.0                     # association radius, px
    n_mon: int = 31                          # monitoring steps after last detection
    t_bf: int = 32                           # backward-fill steps
    ring_len: int = 64                       # dynamic-spectrum window = CNN input width
    qc_band_z: float = 5.0                   # App. A: threshold "of e.g. 5"
    qc_rms_z: float = 5.0                    # same test on band RMS; <= 0 disables
    qc_rms_floor: float = 0.05               # RMS scale floor, fraction of the median RMS
    qc_pixel_zeta: float = 30.0              # App. A leaves the value open
    qc_warmup: int = 8                       # accepted frames before the zeta test arms
    max_sources: int = 8192
    peak_cap: int = 512                      # per band and frame
    prefilter_sigma: float = 0.0             # > 0: detect on the image correlated with a Gaussian PSF of this width
    prefilter_k: int = 0                     # its half-width; <= 0: ceil(4 sigma)
    flux_bg_width: int = 0                   # > 0: flux minus the mean of an annulus this wide around the box

    def __post_init__(self):
        if self.k_bg <= 0:
            self.k_bg = int(math.ceil(3.0 * self.s))
        if self.prefilter_sigma > 0 and self.prefilter_k <= 0:
            self.prefilter_k = int(math.ceil(4.0 * self.prefilter_sigma))
        if self.freqs_mhz is None:
            self.freqs_mhz = np.linspace(60.0, 70.0, self.B)

    @property
    def mask(self) -> np.ndarray:
        if self.sky_mask is None:
            return np.ones((self.H, self.W), dtype=bool)
        return np.asarray(self.sky_mask).astype(bool)

    def grid_row(self, b: int) -> int:
        """Row of band b in the 16-row network input grid (bands ascending)."""
        return b * (16 // self.B)
