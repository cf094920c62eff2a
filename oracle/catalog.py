"""Source association and monitoring (Sec. 2.2).

At step t the per-band peak lists are merged:
1. duplicates of one source seen in several bands are removed: peaks are
   visited in order of decreasing pixel value x (ties: lower band, row,
   column first) and a peak is kept unless it lies within r_dup (Euclidean,
   pixels) of an already kept peak;
2. each kept peak, in the same order, is matched to the nearest live source
   of the catalogue within r_assoc that no earlier peak matched this step
   (distance ties: lower id); a match refreshes the source's last-detection
   step, otherwise a new source is opened at the peak's pixel (ids count up
   in this order); when max_sources sources are held the peak is dropped
   and counted;
3. a source is measured while t - t_last_det <= n_mon; its episode ends with
   the step t_end = t_last_det + n_mon, after which it is reported as ended
   once and released at the following step.
Readings: distances in pixels (no sky coordinates), positions fixed at first
detection; the representative of duplicates is the brightest raw value.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np


@dataclasses.dataclass
class SourceRec:
    id: int
    row: int
    col: int
    t_first: int
    t_last_det: int
    t_end: int = -1          # set when the episode ends
    ended: bool = False


def priority_order(peaks: List[tuple]) -> List[int]:
    """Indices of peaks sorted by (x desc, b asc, i asc, j asc); x compared
    as the float32 pixel value it is."""
    keys = [(-np.float32(p[3]), p[0], p[1], p[2]) for p in peaks]
    return sorted(range(len(peaks)), key=lambda n: keys[n])


def dedupe(peaks: List[tuple], r_dup: float) -> List[int]:
    """Indices (in priority order) of the peaks kept after duplicate removal."""
    kept: List[int] = []
    r2 = r_dup * r_dup
    for n in priority_order(peaks):
        _, i, j = peaks[n][0], peaks[n][1], peaks[n][2]
        if any((i - peaks[m][1]) ** 2 + (j - peaks[m][2]) ** 2 <= r2 for m in kept):
            continue
        kept.append(n)
    return kept


class Catalog:
    def __init__(self, max_sources: int, n_mon: int, r_dup: float, r_assoc: float):
        self.max_sources = max_sources
        self.n_mon = n_mon
        self.r_dup = r_dup
        self.r_assoc = r_assoc
        self.sources: Dict[int, SourceRec] = {}
        self.next_id = 0

    def step(self, t: int, peaks: List[tuple]):
        """Run one step.  Returns (new_ids, ended_ids, measured_ids, dropped)."""
        # release the episodes reported as ended at an earlier step
        for sid in [s for s, r in self.sources.items() if r.ended]:
            del self.sources[sid]
        ended: List[int] = []
        # a gap in t can carry a source past its last measured step
        for r in self.sources.values():
            if t - r.t_last_det > self.n_mon:
                r.ended = True
                r.t_end = r.t_last_det + self.n_mon
                ended.append(r.id)
        live = [r for r in self.sources.values() if not r.ended]
        kept = dedupe(peaks, self.r_dup)
        matched = set()
        new_ids: List[int] = []
        dropped = 0
        ra2 = self.r_assoc * self.r_assoc
        for n in kept:
            _, i, j = peaks[n][0], peaks[n][1], peaks[n][2]
            best: Tuple[int, int] = None
            for r in live:
                if r.id in matched:
                    continue
                d2 = (i - r.row) ** 2 + (j - r.col) ** 2
                if d2 <= ra2 and (best is None or (d2, r.id) < best):
                    best = (d2, r.id)
            if best is not None:
                matched.add(best[1])
                self.sources[best[1]].t_last_det = t
                continue
            if len(self.sources) >= self.max_sources:
                dropped += 1
                continue
            sid = self.next_id
            self.next_id += 1
            self.sources[sid] = SourceRec(sid, i, j, t, t)
            new_ids.append(sid)
        measured = []
        for r in sorted(self.sources.values(), key=lambda r: r.id):
            if r.ended:
                continue
            measured.append(r.id)
            if t - r.t_last_det == self.n_mon:
                r.ended = True
                r.t_end = t
                ended.append(r.id)
        return new_ids, sorted(ended), measured, dropped
