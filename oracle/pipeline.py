"""One image stream through the hot path, step by step (Fig. 2 order:
quality control -> source detection -> association -> flux -> inference).

Call order per step: ``ingest(t, cube)`` -> ``detect()`` -> ``extract_flux()``;
``infer()`` may follow for the episodes that ended at this step.  Steps must
strictly increase; a gap leaves the skipped steps missing.
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from . import cnn as cnn_mod
from .catalog import Catalog
from .config import OracleConfig
from .detect import band_peaks
from .filters import kernel_taps, prefilter, taps_1d
from .flux import measure, window
from .qc import RunningStats, band_reject


class OracleStream:
    def __init__(self, cfg: OracleConfig):
        self.cfg = cfg
        self.M = cfg.mask
        self.g = kernel_taps(cfg.kernel, cfg.s, cfg.k_bg)
        # optional matched pre-filter: detection runs on the image correlated with the PSF
        self.g_psf = (taps_1d(0, cfg.prefilter_sigma, cfg.prefilter_k) if cfg.prefilter_sigma > 0 else None)
        self.stats = RunningStats(cfg.B, cfg.H, cfg.W)
        self.catalog = Catalog(cfg.max_sources, cfg.n_mon, cfg.r_dup, cfg.r_assoc)
        self.cache: Dict[int, np.ndarray] = {}       # step -> quality-controlled cube
        self.rejected: Dict[int, int] = {}           # step -> band bitmask
        self.series: Dict[int, Dict[int, tuple]] = {}  # id -> {step: (flux, valid)}
        self.t: Optional[int] = None
        self.t_start: Optional[int] = None
        self.last: dict = {}

    # -- step 1: quality control (App. A) -----------------------------------------------
    def ingest(self, t: int, cube: np.ndarray) -> int:
        c = self.cfg
        if self.t is not None and t <= self.t:
            raise ValueError("t must increase")
        cube = np.asarray(cube, dtype=np.float32)
        rej, mean, rms, zm, zr = band_reject(cube, c.qc_band_z, c.qc_rms_z, c.qc_rms_floor)
        zeta = np.zeros(c.B)
        for b in range(c.B):
            if rej >> b & 1:
                continue
            zeta[b] = self.stats.zeta_max(b, cube[b], self.M, c.qc_warmup)
            if zeta[b] > c.qc_pixel_zeta:
                rej |= 1 << b
        clean = cube.copy()
        for b in range(c.B):
            if rej >> b & 1:
                clean[b] = 0.0
            else:
                self.stats.update(b, cube[b])
        self.t = t
        if self.t_start is None:
            self.t_start = t
        self.cache[t] = clean
        self.rejected[t] = rej
        for old in [s for s in self.cache if s < t - c.t_bf]:
            del self.cache[old]
            del self.rejected[old]
        self.last = dict(t=t, rejected=rej, mean=mean, rms=rms, z_mean=zm, z_rms=zr, zeta=zeta)
        return rej

    # -- step 2 + 3: detection, association (Sec. 2.1, 2.2) ------------------------------
    def detection_image(self, t=None):
        """The cube detection runs on at step t: the quality-controlled cube,
        or its PSF-correlated form when the pre-filter is on, rounded to
        float32 as the device stores it, so that the local-maximum test
        compares the same kind of values on both sides."""
        X = self.cache[self.t if t is None else t]
        if self.g_psf is None:
            return X
        return np.stack([prefilter(X[b], self.M, self.g_psf) for b in range(X.shape[0])]).astype(np.float32)

    def find_peaks(self):
        """Peak records of every accepted band of the current step (Sec. 2.1),
        and the bitmask of bands whose list exceeded peak_cap (dropped whole)."""
        c = self.cfg
        X = self.detection_image()
        rej = self.rejected[self.t]
        peaks: List[tuple] = []
        overflow = 0
        for b in range(c.B):
            if rej >> b & 1:
                continue   # an all-zero image has S = 0 and no detections
            recs, _, _, _ = band_peaks(b, X[b], self.M, self.g, c.kappa, c.n_iter, c.k_peak)
            if len(recs) > c.peak_cap:
                overflow |= 1 << b   # a band with too many peaks is dropped whole
                continue
            peaks.extend(recs)
        return peaks, overflow

    def associate(self, peaks: List[tuple], overflow: int = 0):
        """Duplicate removal, association and monitoring (Sec. 2.2) of a peak
        list of the current step."""
        new_ids, ended_ids, measured, dropped = self.catalog.step(self.t, peaks)
        self.last.update(peaks=peaks, new=new_ids, ended=ended_ids, measured=measured,
                         dropped=dropped, overflow=overflow)
        return peaks, new_ids, ended_ids

    def detect(self):
        return self.associate(*self.find_peaks())

    # -- step 4: flux + backward fill (Sec. 2.2) ------------------------------------------
    def extract_flux(self):
        c = self.cfg
        t = self.t
        for sid in self.last["measured"]:
            r = self.catalog.sources[sid]
            self._record(sid, t, r.row, r.col)
        for sid in self.last["new"]:
            r = self.catalog.sources[sid]
            for tau in range(max(t - c.t_bf, self.t_start), t):
                if tau in self.cache:
                    self._record(sid, tau, r.row, r.col)

    def _record(self, sid: int, tau: int, i: int, j: int):
        c = self.cfg
        f = measure(self.cache[tau], i, j, c.k_flux, c.flux_bg_width)
        rej = self.rejected[tau]
        v = np.array([not (rej >> b & 1) for b in range(c.B)])
        self.series.setdefault(sid, {})[tau] = (f, v)

    # -- step 5: inference (Sec. 2.3) ------------------------------------------------------
    def spectrum(self, sid: int):
        """(grid [16][ring_len], valid [B][ring_len]) of source sid."""
        c = self.cfg
        r = self.catalog.sources[sid]
        t_end = r.t_end if r.ended else self.t
        rows = [c.grid_row(b) for b in range(c.B)]
        return window(self.series.get(sid, {}), t_end, c.B, c.ring_len, rows)

    def infer(self, wts: dict, ids: Optional[List[int]] = None):
        """(mu [N][4], L [N][10], ids) for the given ids or the episodes that
        ended at the current step."""
        if ids is None:
            ids = list(self.last.get("ended", []))
        if not ids:
            return np.zeros((0, 4)), np.zeros((0, 10)), []
        x = np.stack([self.spectrum(s)[0] for s in ids])
        mu, L = cnn_mod.forward(x, wts)
        return mu, L, list(ids)
