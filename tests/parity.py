"""Helpers shared by the device-vs-oracle parity tests.

Tolerances (FP32 device path vs the FP64 oracle):
* centre C:  |C_dev - C| <= 1e-5 (G*(W|X|)) / (G*W)        (scale-aware: C ~ 0 on noise)
* spread S:  |S_dev - S| <= 1e-5 (G*(W(|X| + |C|)^2)) / (G*W)
* peaks (one clip iteration): with sig = (x - c) / sqrt(s) from the oracle,
  every local maximum with sig > kappa + 1e-3 is listed and nothing with
  sig <= kappa - 1e-3 is; each listed record's sig within 1e-5 (1 + |sig|)
  (x, band, row, col exact; the threshold is monotone in kappa, so this is
  the bracketing P(kappa + d) <= P_dev <= P(kappa - d));
* QC band statistics: float64 on both sides, 1e-12 relative; decisions
  identical unless a score is within 1e-5 (relative) of its threshold;
* Welford state: 1e-5 of the pixel's RMS (mean) / sum of squares (M2);
* fluxes and dynamic spectra: bitwise identical (pure selection);
* network: per output 1e-5 of the last layer's condition scale given exact
  inputs, |W_fc2| |h| + |b_fc2| with h the oracle's hidden activations (the
  same for the softplus diagonal, whose slope is below one).
"""

from __future__ import annotations

import numpy as np

from oracle.config import OracleConfig
from oracle.filters import centre_spread, correlate_2d
from oracle.pipeline import OracleStream

PARAM_MAP = dict(kappa="kappa", bg_sigma="s", bg_halfwidth="k_bg", kernel="kernel",
                 clip_iters="n_iter", peak_halfwidth="k_peak", flux_halfwidth="k_flux",
                 dup_radius="r_dup", assoc_radius="r_assoc", monitor_steps="n_mon",
                 backfill_steps="t_bf", qc_band_z="qc_band_z", qc_rms_z="qc_rms_z",
                 qc_rms_floor="qc_rms_floor", qc_pixel_zeta="qc_pixel_zeta",
                 qc_warmup="qc_warmup", max_sources="max_sources", peak_cap="peak_cap",
                 psf_sigma="prefilter_sigma", psf_halfwidth="prefilter_k", flux_bg_width="flux_bg_width")
DEVICE_ONLY = ("debug_planes", "filter_precision")
FLOAT_PARAMS = ("kappa", "bg_sigma", "dup_radius", "assoc_radius", "qc_band_z", "qc_rms_z", "qc_rms_floor",
                "qc_pixel_zeta", "psf_sigma")


def make_pair(B, H, W, sky_mask=None, grid_rows=None, **params):
    """(device Context, OracleStream) with the same parameters."""
    from paper_2103_15418_amd import Context
    ctx = Context(B, H, W, sky_mask=sky_mask, grid_rows=grid_rows, **params)
    ok = {PARAM_MAP[k]: v for k, v in params.items() if k in PARAM_MAP}
    if "k_bg" in ok and ok["k_bg"] <= 0:
        ok.pop("k_bg")
    ocfg = OracleConfig(B=B, H=H, W=W, sky_mask=sky_mask, **ok)
    # the C configuration holds these parameters as float32: the oracle gets
    # the same values (e.g. 0.05 becomes 0.0500000007..., which moves a
    # floored RMS z by 1.5e-8 relative)
    for key in FLOAT_PARAMS:
        setattr(ocfg, PARAM_MAP[key], float(np.float32(getattr(ctx.cfg, key))))
    if grid_rows is not None:
        rows = list(grid_rows)
        ocfg.grid_row = lambda b, rows=rows: rows[b]
    return ctx, OracleStream(ocfg)


def check_planes(Cd, Sd, X, M, g, rej, label=""):
    """Dense C / S planes of one step (one clip iteration) against the oracle."""
    for b in range(X.shape[0]):
        if rej >> b & 1:
            continue
        C, S, den = centre_spread(X[b], M, g)
        w = M.astype(np.float64)
        pos = den > 0
        safe = np.where(pos, den, 1.0)
        scC = np.where(pos, correlate_2d(w * np.abs(X[b].astype(np.float64)), g) / safe, 0.0)
        scS = np.where(pos, correlate_2d(w * (np.abs(X[b].astype(np.float64)) + np.abs(C)) ** 2, g) / safe, 0.0)
        eC = np.abs(Cd[b].astype(np.float64) - C)
        eS = np.abs(Sd[b].astype(np.float64) - S)
        bad_c = eC > 1e-5 * scC + 1e-30
        bad_s = eS > 1e-5 * scS + 1e-30
        assert not bad_c.any(), (label, b, "C", float((eC / np.maximum(scC, 1e-30)).max()))
        assert not bad_s.any(), (label, b, "S", float((eS / np.maximum(scS, 1e-30)).max()))


def oracle_sig_map(Xb, M, g, k_peak):
    """(Q local-max map, sig = (x - c)/sqrt(s) or +-inf) for one band, one iteration."""
    from oracle.detect import local_max
    C, S, den = centre_spread(Xb, M, g)
    x = Xb.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        sig = np.where(S > 0, (x - C) / np.sqrt(S), np.where(x > C, np.inf, -np.inf))
    sig = np.where(M & (den > 0), sig, -np.inf)
    return local_max(Xb, M, k_peak), sig, C, S


def check_peaks_bracket(peaks_dev, X, M, g, kappa, k_peak, rej, label="", delta=1e-3):
    """Bracketing rule at one clip iteration; returns the number of excused differences."""
    dev = {(int(p["band"]), int(p["row"]), int(p["col"])): p for p in peaks_dev}
    excused = 0
    for b in range(X.shape[0]):
        if rej >> b & 1:
            assert not any(k[0] == b for k in dev), (label, "peaks in a rejected band")
            continue
        Q, sig, C, S = oracle_sig_map(X[b], M, g, k_peak)
        must = Q & (sig > kappa + delta)
        may = Q & (sig > kappa - delta)
        got = np.zeros_like(Q)
        for (bb, i, j), p in dev.items():
            if bb != b:
                continue
            got[i, j] = True
            assert may[i, j], (label, b, i, j, float(sig[i, j]))
            assert p["x"] == np.float32(X[b, i, j])
            s_or = sig[i, j]
            if np.isfinite(s_or):
                assert abs(float(p["sig"]) - s_or) <= 1e-5 * (1 + abs(s_or)), (label, b, i, j)
        missing = must & ~got
        assert not missing.any(), (label, b, np.argwhere(missing)[:5].tolist())
        excused += int((got ^ (Q & (sig > kappa))).sum())
    return excused


def cnn_scale(x, wts):
    """Per raw output: |W_fc2| |h| + |b_fc2|, h = FP64 hidden activations of the oracle.

    (Propagating |W| |x| through every layer instead grows geometrically with
    depth and would make any tolerance vacuous.)"""
    from oracle import cnn
    a = np.asarray(x, dtype=np.float64)
    if a.ndim == 3:
        a = a[:, None]
    alpha = float(wts.get("alpha", 0.0))
    for l in range(1, 5):
        a = cnn.act(cnn.conv3x3(a, wts[f"conv{l}.w"], wts[f"conv{l}.b"]), alpha)
    h = cnn.act(a.reshape(a.shape[0], -1) @ np.asarray(wts["fc1.w"], np.float64).T
                + np.asarray(wts["fc1.b"], np.float64), alpha)
    return np.abs(h) @ np.abs(np.asarray(wts["fc2.w"], np.float64)).T + np.abs(np.asarray(wts["fc2.b"], np.float64))


# ---------------------------------------------------------------------------
# Several clip iterations (Sec. 2.1.1 repeat, App. C)
# ---------------------------------------------------------------------------

def _dilate(mask, r):
    """Chebyshev dilation of a boolean plane by r pixels."""
    if r <= 0 or not mask.any():
        return mask.copy()
    from scipy import ndimage
    return ndimage.maximum_filter(mask.astype(np.uint8), size=2 * r + 1, mode="constant") > 0


def clip_reference(Xb, M, g, kappa, n_iter, k_bg, delta=1e-3):
    """Oracle iterations of one band with the zones where a device in FP32 may
    legitimately differ.

    A pixel is fragile in iteration i when it is a candidate (in the mask,
    G*W > 0, not yet clipped) and its margin (x - c)/sqrt(s) - kappa is within
    delta of zero.  Its decision can flip; the flip changes W of iteration
    i + 1, hence C within k_bg and S within 2 k_bg of it, and so on for every
    later iteration.  Returns dict(Y, C, S, den, W (weights of the last
    iteration), iters, n_fragile, zoneY (Y may differ), zoneCS (C, S may
    differ))."""
    from oracle.detect import sigma_clip
    trace = []
    Y, C, S, den, it = sigma_clip(Xb, M, g, kappa, n_iter, trace=trace)
    x = np.asarray(Xb, dtype=np.float64)
    zoneY = np.zeros(x.shape, dtype=bool)
    n_frag = 0
    for i, (Yb, Ci, Si, di) in enumerate(trace, start=1):
        cand = M & (di > 0) & ~Yb & (Si > 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            marg = np.where(cand, (x - Ci) / np.sqrt(np.where(Si > 0, Si, 1.0)) - kappa, np.inf)
        frag = cand & (np.abs(marg) < delta)
        if frag.any():
            n_frag += int(frag.sum())
            zoneY |= _dilate(frag, 2 * k_bg * (n_iter - i))
    zoneCS = _dilate(zoneY, 2 * k_bg) if zoneY.any() else zoneY
    Wlast = M & ~trace[-1][0]
    return dict(Y=Y, C=C, S=S, den=den, W=Wlast, iters=it, n_fragile=n_frag, zoneY=zoneY, zoneCS=zoneCS)


def check_clip_band(ref, Yd, Cd, Sd, Xb, g, label=""):
    """Device Y, C, S of one band against clip_reference outside its zones."""
    keep = ~ref["zoneY"]
    dY = (Yd.astype(bool) != ref["Y"]) & keep
    assert not dY.any(), (label, "Y", np.argwhere(dY)[:5].tolist())
    w = ref["W"].astype(np.float64)
    den = ref["den"]
    pos = (den > 0) & ~ref["zoneCS"]
    safe = np.where(den > 0, den, 1.0)
    xa = np.abs(np.asarray(Xb, dtype=np.float64))
    scC = correlate_2d(w * xa, g) / safe
    scS = correlate_2d(w * (xa + np.abs(ref["C"])) ** 2, g) / safe
    eC = np.abs(Cd.astype(np.float64) - ref["C"])
    eS = np.abs(Sd.astype(np.float64) - ref["S"])
    bad_c = pos & (eC > 1e-5 * scC + 1e-30)
    bad_s = pos & (eS > 1e-5 * scS + 1e-30)
    assert not bad_c.any(), (label, "C", float((eC / np.maximum(scC, 1e-30))[pos].max()))
    assert not bad_s.any(), (label, "S", float((eS / np.maximum(scS, 1e-30))[pos].max()))


def check_peaks_iters(peaks_dev, refs, X, M, k_peak, label=""):
    """Peaks after several iterations: P = Q and Y, identical to the oracle's
    outside the zones where Y may differ; inside them every listed pixel must
    be a local maximum with a valid record.  refs: {band: clip_reference}.
    Returns the number of differences inside zones."""
    from oracle.detect import local_max
    dev = {}
    for p in peaks_dev:
        dev[(int(p["band"]), int(p["row"]), int(p["col"]))] = p
    excused = 0
    for b, ref in refs.items():
        Q = local_max(X[b], M, k_peak)
        P = Q & ref["Y"]
        got = np.zeros_like(P)
        for (bb, i, j), p in dev.items():
            if bb == b:
                got[i, j] = True
                assert Q[i, j], (label, b, i, j, "not a local maximum")
                assert p["x"] == np.float32(X[b, i, j]), (label, b, i, j)
                if not ref["zoneCS"][i, j]:
                    c, s = ref["C"][i, j], ref["S"][i, j]
                    assert abs(float(p["c"]) - c) <= 1e-5 * (1 + abs(c) + np.sqrt(max(s, 0.0))), (label, b, i, j)
                    if s > 0:
                        sig = (float(np.float32(X[b, i, j])) - c) / np.sqrt(s)
                        assert abs(float(p["sig"]) - sig) <= 1e-5 * (1 + abs(sig)) + 1e-4, (label, b, i, j)
        diff = got ^ P
        assert not (diff & ~ref["zoneY"]).any(), (label, b, np.argwhere(diff & ~ref["zoneY"])[:5].tolist())
        excused += int(diff.sum())
    bands = {k[0] for k in dev}
    assert bands <= set(refs), (label, "peaks in a band that was not detected", bands - set(refs))
    return excused


# ---------------------------------------------------------------------------
# Step-by-step stream comparison
# ---------------------------------------------------------------------------

def _key(p):
    return (int(p["band"]), int(p["row"]), int(p["col"]))


def dev_peaks_as_oracle(peaks_dev):
    """Device peak records as the oracle's tuples (b, i, j, x, c, s, sig); the
    association uses (b, i, j) and the float32 value x only."""
    return [(int(p["band"]), int(p["row"]), int(p["col"]), float(p["x"]), float(p["c"]),
             float(p["s"]), float(p["sig"])) for p in sorted(peaks_dev, key=_key)]


def compare_events(ev, orc, new_o, ended_o, label):
    """Device events of the step against the oracle's, exactly: new (id
    order) then ended (id order), positions and times."""
    exp = [(sid, 1) for sid in new_o] + [(sid, 2) for sid in ended_o]
    got = [(int(e["id"]), int(e["event"])) for e in ev]
    assert got == exp, (label, got[:8], exp[:8])
    for e in ev:
        r = orc.catalog.sources[int(e["id"])]
        assert (int(e["row"]), int(e["col"])) == (r.row, r.col), label
        assert int(e["t_first"]) == r.t_first and int(e["t_last_det"]) == r.t_last_det, label
        if e["event"] == 2:
            assert int(e["t_end"]) == r.t_end, label


def _event_rows(orc_catalog, ids, kind):
    return [(kind, orc_catalog.sources[s].row, orc_catalog.sources[s].col,
             orc_catalog.sources[s].t_first, orc_catalog.sources[s].t_last_det) for s in ids]


def check_events_excused(orc, own_peaks, dev_peaks_o, overflow, excused_pos, label):
    """At a step where the device's peak list differs from the oracle's at
    excused pixels only: the events the oracle derives from its own list and
    those it derives from the device's list may differ only at sources within
    r_dup + r_assoc of an excused pixel (a peak there can take over a
    duplicate or an association of a neighbour).  Compared as (kind, row,
    col, t_first, t_last_det) rows, ids aside (ids count up in greedy order,
    so one extra source shifts later ids)."""
    import copy
    c = orc.cfg
    rad = c.r_dup + c.r_assoc
    res = []
    for plist in (own_peaks, dev_peaks_o):
        cat = copy.deepcopy(orc.catalog)
        new, ended, _, _ = cat.step(orc.t, plist)
        res.append(sorted(_event_rows(cat, new, 1) + _event_rows(cat, ended, 2)))

    def far(row):
        return all((row[1] - i) ** 2 + (row[2] - j) ** 2 > rad * rad for (i, j) in excused_pos)
    a = [r for r in res[0] if far(r)]
    b = [r for r in res[1] if far(r)]
    assert a == b, (label, "events differ away from excused peaks", a[:6], b[:6])


def run_steps(ctx, orc, frames, ts, compare_planes=False, label="", spectra=64, qc_scores=True,
              on_step=None):
    """Runs the device context and the oracle over the frames and compares
    every stage at every step:

    * QC: band mean / RMS (float64, 1e-12), robust z of both (float64, 1e-9
      relative), max |zeta| of armed bands that passed the band tests (float32
      state on the device: 1e-5 relative), decisions (identical unless a score
      is within 1e-5 of its threshold: then the run stops comparing, since the
      caches differ from there on);
    * peaks: bracketing at one clip iteration, the zone rule of
      check_peaks_iters at several;
    * events: exact.  Where the peak lists differ at excused pixels, the
      oracle's own events are compared with those it derives from the device
      list away from the excused pixels, and the oracle then continues from
      the device list, so that every later step is again compared exactly;
    * dynamic spectra of up to ``spectra`` held sources: bitwise.
    Returns counters."""
    stats = dict(steps=0, excused=0, resyncs=0, events=0, spectra=0, zeta_checked=0, fragile=0, rc=[])
    g, M = orc.g, orc.M
    c = orc.cfg
    for t, cube in zip(ts, frames):
        print(f"{label} step t={t}", flush=True)
        rej_o = orc.ingest(t, cube)
        rej_d = ctx.ingest(t, cube, want_rejected=True)
        bs = ctx.debug_read("bandstats")
        L = orc.last
        n_before = orc.stats.n.copy()
        for b in range(ctx.B):
            if not np.isfinite(L["rms"][b]):
                assert bs[b, 5] > 0 and (rej_d >> b & 1), (label, t, b)
                continue
            assert abs(bs[b, 0] - L["mean"][b]) <= 1e-12 * max(1.0, abs(L["rms"][b])), (label, t, b)
            assert abs(bs[b, 1] - L["rms"][b]) <= 1e-12 * max(1.0, L["rms"][b]), (label, t, b)
            if qc_scores:
                for col, key in ((2, "z_mean"), (3, "z_rms")):
                    zo = L[key][b]
                    if np.isfinite(zo):
                        assert abs(bs[b, col] - zo) <= 1e-9 * max(1.0, abs(zo)), (label, t, b, key, bs[b, col], zo)
                zo = L["zeta"][b]
                if zo > 0 and np.isfinite(zo):
                    assert abs(bs[b, 4] - zo) <= 1e-5 * zo, (label, t, b, "zeta", bs[b, 4], zo)
                    stats["zeta_checked"] += 1
        if rej_o != rej_d:
            for b in range(ctx.B):
                if (rej_o ^ rej_d) >> b & 1:
                    near = (abs(abs(L["z_mean"][b]) - c.qc_band_z) <= 1e-5 * c.qc_band_z
                            or abs(abs(L["z_rms"][b]) - c.qc_rms_z) <= 1e-5 * c.qc_rms_z
                            or abs(L["zeta"][b] - c.qc_pixel_zeta) <= 1e-5 * c.qc_pixel_zeta)
                    assert near, (label, t, b, rej_o, rej_d)
            stats["qc_diverged_at"] = t
            return stats
        X = orc.cache[t]
        pd, ev, rc = ctx.detect()
        own, overflow = orc.find_peaks()
        if c.n_iter == 1:
            if compare_planes:
                check_planes(ctx.debug_read("centre"), ctx.debug_read("spread"), X, M, g, rej_o, label)
            ok_bands = ~np.array([(rej_o | overflow) >> b & 1 for b in range(ctx.B)], dtype=bool)
            ex = check_peaks_bracket([p for p in pd if ok_bands[int(p["band"])]], X, M, g, c.kappa, c.k_peak,
                                     rej_o | overflow, f"{label} t={t}")
        else:
            Yd = ctx.debug_read("clipmask")
            Cd = ctx.debug_read("centre")
            Sd = ctx.debug_read("spread")
            refs = {}
            for b in range(ctx.B):
                if rej_o >> b & 1:
                    continue
                refs[b] = clip_reference(X[b], M, g, c.kappa, c.n_iter, c.k_bg)
                stats["fragile"] += refs[b]["n_fragile"]
                check_clip_band(refs[b], Yd[b], Cd[b], Sd[b], X[b], g, f"{label} t={t} b={b}")
            refs_ok = {b: r for b, r in refs.items() if not (overflow >> b & 1)}
            ex = check_peaks_iters([p for p in pd if int(p["band"]) in refs_ok], refs_ok, X, M, c.k_peak,
                                   f"{label} t={t}")
        st = ctx.status()
        assert st["overflow_bands"] == overflow, (label, t, st["overflow_bands"], overflow)
        stats["rc"].append(rc)
        stats["excused"] += ex
        dev_list = [p for p in pd if not (overflow >> int(p["band"]) & 1)]
        same = sorted(_key(p) for p in dev_list) == sorted((p[0], p[1], p[2]) for p in own)
        if same:
            peaks_use = own
        else:
            dset = {_key(p) for p in dev_list}
            oset = {(p[0], p[1], p[2]) for p in own}
            excused_pos = [(i, j) for (_, i, j) in dset ^ oset]
            dev_o = dev_peaks_as_oracle(dev_list)
            check_events_excused(orc, own, dev_o, overflow, excused_pos, f"{label} t={t}")
            peaks_use = dev_o
            stats["resyncs"] += 1
        _, new_o, ended_o = orc.associate(peaks_use, overflow)
        compare_events(ev, orc, new_o, ended_o, f"{label} t={t}")
        assert st["n_dropped"] == orc.last["dropped"], (label, t, st["n_dropped"], orc.last["dropped"])
        assert st["n_new"] == len(new_o) and st["n_ended"] == len(ended_o), (label, t)
        stats["events"] += len(ev)
        orc.extract_flux()
        ctx.extract_flux()
        stats["steps"] += 1
        held = list(orc.catalog.sources)
        if len(held) > spectra:
            rng = np.random.default_rng(t)
            held = sorted(rng.choice(held, spectra, replace=False).tolist())
        rows = [c.grid_row(b) for b in range(ctx.B)]
        for sid in held:
            grid, valid = orc.spectrum(sid)
            out, vd, tl = ctx.read_spectrum(sid)
            assert np.array_equal(vd, valid), (label, t, sid)
            exp_vals = np.where(valid, grid[rows, :], 0.0).astype(np.float32)
            assert np.array_equal(out, exp_vals), (label, t, sid)
            stats["spectra"] += 1
        if on_step is not None:
            on_step(t, stats)
    return stats


# ---------------------------------------------------------------------------
# Full-size images: outputs the oracle computes one by one
# ---------------------------------------------------------------------------

def local_estimates(Xb, M, g, i, j, k_bg):
    """(C, S, den) at pixel (i, j) from the oracle on the window of radius
    2 k_bg around it: C there uses x within k_bg, S uses C within k_bg, so the
    window gives the full-image values exactly (the image edge is the
    window's edge where they meet)."""
    H, W = Xb.shape
    r = 2 * k_bg
    r0, r1 = max(0, i - r), min(H, i + r + 1)
    c0, c1 = max(0, j - r), min(W, j + r + 1)
    C, S, den = centre_spread(Xb[r0:r1, c0:c1], M[r0:r1, c0:c1], g)
    return C[i - r0, j - c0], S[i - r0, j - c0], den[i - r0, j - c0]


def _is_local_max(Xb, M, i, j, k):
    H, W = Xb.shape
    if not M[i, j]:
        return False
    r0, r1 = max(0, i - k), min(H, i + k + 1)
    c0, c1 = max(0, j - k), min(W, j + k + 1)
    win = np.where(M[r0:r1, c0:c1], Xb[r0:r1, c0:c1].astype(np.float64), -np.inf)
    return float(Xb[i, j]) == float(win.max())


def check_peaks_sampled(peaks_dev, X, M, g, kappa, k_peak, k_bg, rej, rng, n_tiles=2, tile=256,
                        label="", delta=1e-3):
    """One clip iteration at full size.  Validity of every listed peak (a
    local maximum of the window within the image and the mask, margin above
    -delta, record values at the tolerance), computed pixel by pixel; and
    completeness on n_tiles random tiles per accepted band: every local
    maximum there with margin above +delta is listed.  Returns the number of
    listed peaks whose margin lies within delta of the threshold."""
    B, H, W = X.shape
    by_band = {}
    near = 0
    for p in peaks_dev:
        b, i, j = _key(p)
        assert not (rej >> b & 1), (label, "peak in a rejected band", b)
        by_band.setdefault(b, set()).add((i, j))
        assert p["x"] == np.float32(X[b, i, j]), (label, b, i, j)
        assert _is_local_max(X[b], M, i, j, k_peak), (label, b, i, j, "not a local maximum")
        C, S, den = local_estimates(X[b], M, g, i, j, k_bg)
        assert den > 0, (label, b, i, j)
        sig = (float(np.float32(X[b, i, j])) - C) / np.sqrt(S) if S > 0 else np.inf
        assert sig > kappa - delta, (label, b, i, j, sig)
        if sig < kappa + delta:
            near += 1
        assert abs(float(p["c"]) - C) <= 1e-5 * (1 + abs(C) + np.sqrt(S)), (label, b, i, j, float(p["c"]), C)
        if np.isfinite(sig):
            assert abs(float(p["sig"]) - sig) <= 1e-5 * (1 + abs(sig)), (label, b, i, j, float(p["sig"]), sig)
    from oracle.detect import local_max
    h = 2 * k_bg + k_peak + 1
    for b in range(B):
        if rej >> b & 1:
            continue
        for _ in range(n_tiles):
            ti = int(rng.integers(0, max(1, H - tile + 1)))
            tj = int(rng.integers(0, max(1, W - tile + 1)))
            r0, r1 = max(0, ti - h), min(H, ti + tile + h)
            c0, c1 = max(0, tj - h), min(W, tj + tile + h)
            Xt, Mt = X[b, r0:r1, c0:c1], M[r0:r1, c0:c1]
            C, S, den = centre_spread(Xt, Mt, g)
            Q = local_max(Xt, Mt, k_peak)
            x = Xt.astype(np.float64)
            with np.errstate(divide="ignore", invalid="ignore"):
                sig = np.where(S > 0, (x - C) / np.sqrt(S), np.where(x > C, np.inf, -np.inf))
            must = Q & Mt & (den > 0) & (sig > kappa + delta)
            ii, jj = np.nonzero(must)
            got = by_band.get(b, set())
            for i, j in zip((ii + r0).tolist(), (jj + c0).tolist()):
                if ti <= i < ti + tile and tj <= j < tj + tile:
                    assert (i, j) in got, (label, b, i, j, "missing peak")
    return near


def check_centre_sampled(Cd, X, M, g, k_bg, rej, rng, n=32, label=""):
    """C of the device plane at n random sky pixels against the oracle's
    one-by-one value (scale-aware tolerance of the dense check)."""
    B, H, W = X.shape
    done = 0
    while done < n:
        b = int(rng.integers(B))
        if rej >> b & 1:
            continue
        i, j = int(rng.integers(H)), int(rng.integers(W))
        if not M[i, j]:
            continue
        C, S, den = local_estimates(X[b], M, g, i, j, k_bg)
        r = 2 * k_bg
        r0, r1 = max(0, i - r), min(H, i + r + 1)
        c0, c1 = max(0, j - r), min(W, j + r + 1)
        sc = correlate_2d(M[r0:r1, c0:c1] * np.abs(X[b, r0:r1, c0:c1].astype(np.float64)), g)[i - r0, j - c0] / den
        assert abs(float(Cd[b, i, j]) - C) <= 1e-5 * sc + 1e-30, (label, b, i, j, float(Cd[b, i, j]), C)
        done += 1


def run_steps_sampled(ctx, orc, frame_fn, ts, label="", spectra=64, tiles=2, check_welford_at=(),
                      on_step=None):
    """Full-size form of run_steps: QC statistics and decisions as there;
    peaks by check_peaks_sampled (the oracle's dense detection is not run);
    the oracle's catalogue then continues from the device's validated list,
    so events are compared exactly and dynamic spectra bitwise."""
    stats = dict(steps=0, near=0, events=0, spectra=0, zeta_checked=0, ended=0, peaks=0)
    g, M = orc.g, orc.M
    c = orc.cfg
    rng = np.random.default_rng(12345)
    for t in ts:
        cube = frame_fn(t)
        print(f"{label} step t={t}", flush=True)
        rej_o = orc.ingest(t, cube)
        rej_d = ctx.ingest(t, cube, want_rejected=True)
        bs = ctx.debug_read("bandstats")
        L = orc.last
        for b in range(ctx.B):
            if not np.isfinite(L["rms"][b]):
                continue
            assert abs(bs[b, 0] - L["mean"][b]) <= 1e-12 * max(1.0, abs(L["rms"][b])), (label, t, b)
            assert abs(bs[b, 1] - L["rms"][b]) <= 1e-12 * max(1.0, L["rms"][b]), (label, t, b)
            for col, key in ((2, "z_mean"), (3, "z_rms")):
                zo = L[key][b]
                if np.isfinite(zo):
                    assert abs(bs[b, col] - zo) <= 1e-9 * max(1.0, abs(zo)), (label, t, b, key)
            zo = L["zeta"][b]
            if zo > 0 and np.isfinite(zo):
                assert abs(bs[b, 4] - zo) <= 1e-5 * zo, (label, t, b, "zeta", bs[b, 4], zo)
                stats["zeta_checked"] += 1
        assert rej_o == rej_d, (label, t, rej_o, rej_d)
        X = orc.cache[t]
        pd, ev, rc = ctx.detect()
        st = ctx.status()
        assert st["overflow_bands"] == 0, (label, t, "overflow at full size")
        stats["near"] += check_peaks_sampled(pd, X, M, g, c.kappa, c.k_peak, c.k_bg, rej_o, rng, tiles,
                                             label=f"{label} t={t}")
        check_centre_sampled(ctx.debug_read("centre"), X, M, g, c.k_bg, rej_o, rng, label=f"{label} t={t}")
        stats["peaks"] += len(pd)
        _, new_o, ended_o = orc.associate(dev_peaks_as_oracle(pd), 0)
        compare_events(ev, orc, new_o, ended_o, f"{label} t={t}")
        assert st["n_dropped"] == orc.last["dropped"], (label, t)
        stats["events"] += len(ev)
        stats["ended"] += len(ended_o)
        orc.extract_flux()
        ctx.extract_flux()
        held = list(orc.catalog.sources)
        if len(held) > spectra:
            held = sorted(rng.choice(held, spectra, replace=False).tolist())
        rows = [c.grid_row(b) for b in range(ctx.B)]
        for sid in held:
            grid, valid = orc.spectrum(sid)
            out, vd, tl = ctx.read_spectrum(sid)
            assert np.array_equal(vd, valid), (label, t, sid)
            assert np.array_equal(out, np.where(valid, grid[rows, :], 0.0).astype(np.float32)), (label, t, sid)
            stats["spectra"] += 1
        if t in check_welford_at:
            check_welford(ctx, orc, label=f"{label} t={t}")
        stats["steps"] += 1
        if on_step is not None:
            on_step(t, stats)
    return stats


def check_welford(ctx, orc, label=""):
    """Running mean / M2 of accepted steps: 1e-5 of the pixel's RMS / sum of squares."""
    mean_d = ctx.debug_read("welford_mean")
    m2_d = ctx.debug_read("welford_m2")
    n = orc.stats.n
    assert np.array_equal(ctx.debug_read("welford_n"), n.astype(np.int32)), label
    for b in range(ctx.B):
        ssq = orc.stats.m2[b] + n[b] * orc.stats.mean[b] ** 2
        rms = np.sqrt(ssq / max(1, n[b]))
        assert np.all(np.abs(mean_d[b] - orc.stats.mean[b]) <= 1e-5 * rms + 1e-30), (label, b)
        assert np.all(np.abs(m2_d[b] - orc.stats.m2[b]) <= 1e-5 * ssq + 1e-30), (label, b)
