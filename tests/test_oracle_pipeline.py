"""End-to-end pins of the oracle on synthetic dispersed transients:
recovery of injected sources at known positions and the cold-plasma
nu^-2 dispersion delay read back from the dynamic spectra (Sec. 2, Sec. 3.2)."""

import numpy as np
import pytest

import synth
from oracle.config import OracleConfig
from oracle.pipeline import OracleStream


def run(stream, cfg, T, noise=True):
    orc = OracleStream(cfg)
    per_step = []
    windows = {}
    for t in range(T):
        orc.ingest(t, stream.frame(t, noise=noise))
        peaks, new, ended = orc.detect()
        orc.extract_flux()
        per_step.append(peaks)
        for sid in ended:
            r = orc.catalog.sources[sid]
            windows[sid] = (r.row, r.col, r.t_end, orc.spectrum(sid)[0])
    for sid, r in orc.catalog.sources.items():   # still monitored at the end
        if sid not in windows:
            windows[sid] = (r.row, r.col, orc.t, orc.spectrum(sid)[0])
    return orc, per_step, windows


def tiny_cfg(st):
    s = st.spec
    return OracleConfig(B=s.B, H=s.H, W=s.W, freqs_mhz=st.freqs, kappa=4.5, s=8.0)


def full_cells(st, k):
    """(t, b) cells where source k's boxcar fully covers the frame."""
    s = st.spec
    return [(t, b) for t in range(s.T) for b in range(s.B)
            if st.amplitude(k, t, b) >= st.sources[k].amp - 1e-12]


def test_recovery_noise_free_exact():
    """Noise off: every cell with any pulse flux yields exactly one peak, at
    the source's pixel, and nothing else is found.  (Quality control is
    switched off: with empty bands the robust scale is zero and every band
    holding flux would be discarded.)"""
    st = synth.Stream(synth.spec_tiny())
    cfg = tiny_cfg(st)
    cfg.qc_band_z = np.inf
    cfg.qc_rms_z = 0.0
    cfg.qc_pixel_zeta = np.inf
    orc, per_step, _ = run(st, cfg, st.spec.T, noise=False)
    expect = set()
    for k, src in enumerate(st.sources):
        for t in range(st.spec.T):
            for b in range(st.spec.B):
                if st.amplitude(k, t, b) > 0:
                    expect.add((t, b, int(src.row), int(src.col)))
    got = {(t, p[0], p[1], p[2]) for t, peaks in enumerate(per_step) for p in peaks}
    assert expect and got == expect


@pytest.mark.slow
def test_recovery_with_noise_tiny_stream():
    st = synth.Stream(synth.spec_tiny())
    orc, per_step, _ = run(st, tiny_cfg(st), st.spec.T)
    hits = cells = 0
    for k, src in enumerate(st.sources):
        cells_k = full_cells(st, k)
        found = 0
        for (t, b) in cells_k:
            ok = any(p[0] == b and abs(p[1] - src.row) <= 1 and abs(p[2] - src.col) <= 1
                     for p in per_step[t])
            found += ok
        if len(cells_k) >= 2:
            assert found >= 1, k
        hits += found
        cells += len(cells_k)
    assert cells > 0 and hits / cells >= 0.9


@pytest.mark.slow
def test_dispersion_delay_from_dynamic_spectra():
    """Per-band argmax of a recovered source's spectrum sits at the injected
    arrival floor(t_b) or floor(t_b)+1, t_b = t0 + C_DM DM (nu_b^-2 - nu_max^-2),
    and a least-squares fit of those times on nu^-2 returns DM within 10 %."""
    spec = synth.spec_tiny()
    spec.H = spec.W = 160
    spec.T = 90
    spec.n_sources = 4
    spec.place_box = (30, 130)
    spec.dm = (50.0, 100.0)
    spec.t0 = (5.0, 20.0)
    st = synth.Stream(spec)
    cfg = tiny_cfg(st)
    orc, per_step, windows = run(st, cfg, spec.T)
    x = st.freqs ** -2 - st.freqs.max() ** -2
    checked = 0
    for k, src in enumerate(st.sources):
        mine = [w for w in windows.values()
                if abs(w[0] - src.row) <= 1 and abs(w[1] - src.col) <= 1]
        assert mine, k
        row, col, t_end, grid = max(mine, key=lambda w: w[3].max())
        taus = []
        for b in range(spec.B):
            c = int(np.argmax(grid[cfg.grid_row(b)]))
            tau = t_end - cfg.ring_len + 1 + c
            tb = st.arrivals[k, b]
            assert tau in (int(np.floor(tb)), int(np.floor(tb)) + 1), (k, b, tau, tb)
            taus.append(tau + 0.5)
        slope = np.polyfit(x, np.array(taus), 1)[0]
        dm_fit = slope / synth.C_DM
        assert abs(dm_fit - src.dm) < 0.1 * src.dm, (dm_fit, src.dm)
        checked += 1
    assert checked == spec.n_sources
