#!/usr/bin/env python3
"""Throughput of the transient-detection hot path on one MI355X.

One step = one synthetic image cube of the instrument workload (16 subbands
x 1024 x 1024 in a circular sky mask, 50 dispersed point sources, N(0,1)
noise on a smooth background) taken through every stage: quality control +
image cache, centre/spread filters + threshold + peaks, association, flux +
backward fill, and the network on the episodes that end at that step.
Cubes are generated up front and resident in HBM before timing starts.

The stream is fast-forwarded (untimed) past the first monitoring window,
so that episodes end, and the network runs, inside the timed steps; every
step ingests a distinct cube.

Prints one JSON line: subband-pixels per second (metric of the paper's
real-time claim: a 16 x 1024^2 cube per 1 s step), per-frame latency
percentiles (completion of the flux stage minus arrival, frames arriving at
a fixed cadence), the roofline of the dominant kernel (timed with HIP events
recorded by the library on its stream) and the FP64 oracle's rate on a
bounded sample of the same workload on the host CPU (run in a child process
that never touches the GPU).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CU x 128 lanes-FMA/clk (packed) x 2 x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0    # dense bf16 / fp16 matrix rate
# network FLOPs per window: conv 1->32->32->64->64 on 16x64, dense 65536->128->14
CNN_FLOPS = 2 * (16 * 64 * (32 * 9 + 32 * 32 * 9 + 64 * 32 * 9 + 64 * 64 * 9)) + 2 * (65536 * 128 + 128 * 14)


def _spec(name):
    import synth
    return synth.spec_instrument() if name == "instrument" else synth.spec_tiny()


def make_frames(stream, ts, workers):
    """Cubes of the given steps, generated on host threads (numpy releases the
    GIL in the noise generator; no process is forked)."""
    if workers <= 1:
        return [stream.frame(t) for t in ts]
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(stream.frame, ts))


def _band_peaks_job(args):
    from oracle.detect import band_peaks
    b, X, M, g, kappa, n_iter, k_peak = args
    return band_peaks(b, X, M, g, kappa, n_iter, k_peak)[0]


def cpu_baseline_run(spec_name, n_frames, workers):
    """FP64 oracle on steps 0 .. n_frames-1 of the workload, timed around
    ingest + detect + extract_flux per step: once in one process, once with
    the per-band detection (Sec. 2.1, independent per subband) spread over a
    pool of `workers` processes.  Runs in a process that has not touched the
    GPU (bench.py starts it as a child with --cpu-baseline-only)."""
    import multiprocessing as mp

    import synth
    from oracle.config import OracleConfig
    from oracle.pipeline import OracleStream
    spec = _spec(spec_name)
    st = synth.Stream(spec)
    frames = make_frames(st, range(n_frames), workers)
    px = n_frames * spec.B * spec.H * spec.W

    def fresh():
        return OracleStream(OracleConfig(B=spec.B, H=spec.H, W=spec.W, sky_mask=st.mask, freqs_mhz=st.freqs))

    orc = fresh()
    t0 = time.perf_counter()
    for t, f in enumerate(frames):
        orc.ingest(t, f)
        orc.detect()
        orc.extract_flux()
    dt1 = time.perf_counter() - t0
    out = {"single": {"value": px / dt1, "seconds": dt1, "cores": 1}}
    if workers > 1:
        orc = fresh()
        c = orc.cfg
        with mp.get_context("fork").Pool(workers) as pool:
            t0 = time.perf_counter()
            for t, f in enumerate(frames):
                rej = orc.ingest(t, f)
                X = orc.cache[t]
                jobs = [(b, X[b], orc.M, orc.g, c.kappa, c.n_iter, c.k_peak)
                        for b in range(c.B) if not (rej >> b & 1)]
                peaks, overflow = [], 0
                for recs in pool.map(_band_peaks_job, jobs):
                    if len(recs) > c.peak_cap:
                        overflow |= 1 << recs[0][0]
                    else:
                        peaks.extend(recs)
                orc.associate(peaks, overflow)
                orc.extract_flux()
            dt = time.perf_counter() - t0
            pool.close()
            pool.join()
        out["pool"] = {"value": px / dt, "seconds": dt, "cores": workers}
    return out


def cpu_baseline(args):
    """Starts the oracle timing as a child process (no fork of this GPU
    process) and returns the cpu_baseline object."""
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--workload", args.workload,
           "--cpu-frames", str(args.cpu_frames), "--workers", str(cores)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    res = json.loads(r.stdout.strip().splitlines()[-1])
    spec = _spec(args.workload)
    best = res.get("pool", res["single"])
    return {"value": best["value"], "unit": "subband-px/s", "cores": best["cores"], "kind": "oracle",
            "single_process": {"value": res["single"]["value"], "cores": 1},
            "sample": f"steps 0-{args.cpu_frames - 1} of the {args.workload} workload "
                      f"({spec.B}x{spec.H}x{spec.W}): ingest + detect + extract_flux, numpy float64; "
                      f"value with the per-band detection on {best['cores']} processes "
                      f"({best['seconds']:.1f} s), single process {res['single']['seconds']:.1f} s; "
                      f"host threads available {len(os.sched_getaffinity(0))}"}


def precision_errors(code, st, pool, Context, Model, synth, n_frames=2):
    """Error of the 16-bit form per output against the float32 device path
    (itself within 1e-5 of the FP64 oracle, tests/test_gpu_parity.py; the
    16-bit errors against the FP64 oracle per output are printed by
    tests/test_gpu_precision.py): C in units of the local spread,
    |C16 - C32| / sqrt(S32), and S relative, |S16 - S32| / S32 (all sky
    pixels of every band, step 0); the margin sig - kappa at the peaks both
    forms list on the first n_frames steps; each network output on 64 seeded
    windows as |y16 - y32| / (1 + |y32|).  [max, median] each; plus the
    candidate lists' Jaccard index against the float32 path."""
    import torch
    spec = st.spec
    M = torch.from_numpy(st.mask.astype(bool)).cuda()
    c16 = Context(spec.B, spec.H, spec.W, sky_mask=st.mask, filter_precision=code, debug_planes=1)
    c32 = Context(spec.B, spec.H, spec.W, sky_mask=st.mask, debug_planes=1)
    inter = union = 0
    em = []
    per = {}
    for t in range(n_frames):
        c16.ingest(t, pool[t])
        c32.ingest(t, pool[t])
        p16 = c16.detect()[0]
        p32 = c32.detect()[0]
        if t == 0:
            C16 = torch.from_numpy(c16.debug_read("centre")).cuda()
            S16 = torch.from_numpy(c16.debug_read("spread")).cuda()
            C32 = torch.from_numpy(c32.debug_read("centre")).cuda()
            S32 = torch.from_numpy(c32.debug_read("spread")).cuda()
            sel = M.expand_as(C32) & (S32 > 0)
            eC = ((C16 - C32).abs() / S32.clamp_min(1e-30).sqrt())[sel]
            eS = ((S16 - S32).abs() / S32.clamp_min(1e-30))[sel]
            finite = bool(torch.isfinite(C16[sel]).all() and torch.isfinite(S16[sel]).all())
            per["C"] = [float(eC.max()), float(eC.median())]
            per["S"] = [float(eS.max()), float(eS.median())]
        c16.extract_flux()
        c32.extract_flux()
        d32 = {(int(p["band"]), int(p["row"]), int(p["col"])): float(p["sig"]) for p in p32}
        d16 = {(int(p["band"]), int(p["row"]), int(p["col"])): float(p["sig"]) for p in p16}
        inter += len(d16.keys() & d32.keys())
        union += len(d16.keys() | d32.keys())
        em += [abs(d16[k] - d32[k]) for k in d16.keys() & d32.keys()]
    del c16, c32
    per["margin"] = [float(np.max(em)), float(np.median(em))] if em else None
    wts = synth.cnn_weights()
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    x = torch.randn((64, 16, 64), generator=g, device="cuda", dtype=torch.float32) * 2.0
    y = []
    for prec in (0, code):
        m = Model(wts, precision=prec, max_batch=64)
        mu, L = m.infer_windows(x)
        torch.cuda.synchronize()
        y.append(torch.cat([mu, L], 1))
        del m
    e = (y[1] - y[0]).abs() / (1.0 + y[0].abs())
    names = ["mu_DM", "mu_width", "mu_amplitude", "mu_arrival"] + [f"L{k}" for k in range(10)]
    for k, n in enumerate(names):
        per[n] = [float(e[:, k].max()), float(e[:, k].median())]
    return {"reference": "float32 device path (within 1e-5 of the FP64 oracle)",
            "scale": "[max, median]: C |dC|/sqrt(S32); S |dS|/S32; margin |d sig| at common peaks; "
                     "network |dy|/(1+|y32|) (L: packed Cholesky entries, softplus diagonal)",
            "per_output": per, "planes_finite": finite, "margin_peaks": len(em),
            "candidates_jaccard_vs_fp32": inter / max(1, union), "candidates": [inter, union]}


def serving(args, precision, pools, specs, masks, seconds, cadence_s, jitter_s, seed=0):
    """Serving form: all streams admitted under the HBM budget, frames arriving at
    cadence_s +- jitter_s per stream for `seconds`; returns latency statistics."""
    import threading

    import torch
    import synth
    from paper_2103_15418_amd import Model, Server, now_ns, workspace_size, default_config
    model = Model(synth.cnn_weights(), precision=precision, max_batch=1024)
    budget = int(args.serve_budget_gb * 2 ** 30)
    srv = Server(model, budget)
    sids = [srv.admit(s.B, s.H, s.W, sky_mask=m, filter_precision=precision) for s, m in zip(specs, masks)]
    used, _, _ = srv.usage()
    n_steps = max(1, int(round(seconds / cadence_s)))
    rng = np.random.default_rng(seed)
    t0 = now_ns() + int(0.05e9)
    arrivals = []
    for k, sid in enumerate(sids):
        for t in range(n_steps):
            arrivals.append((t0 + int((t * cadence_s + rng.uniform(-jitter_s, jitter_s)) * 1e9), k, t))
    arrivals.sort()

    def submitter():
        for when, k, t in arrivals:
            while True:
                d = when - now_ns()
                if d <= 0:
                    break
                time.sleep(min(d, 2e6) / 1e9)
            srv.submit(sids[k], t, pools[k][t % len(pools[k])], arrival_ns=when)

    th = threading.Thread(target=submitter)
    wall0 = time.perf_counter()
    th.start()
    th.join()
    srv.drain()
    wall = time.perf_counter() - wall0
    res = srv.poll(cap=len(arrivals) + 16)
    srv.close_all()
    lat = (res["done_ns"] - res["arrival_ns"]) / 1e6
    px = sum(specs[int(r["stream_id"])].B * specs[int(r["stream_id"])].H * specs[int(r["stream_id"])].W
             for r in res)
    return {"streams": len(sids), "frames": int(len(res)), "cadence_s": cadence_s, "jitter_s": jitter_s,
            "seconds": seconds, "errors": int(np.sum(res["status"] != 0)),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "deadline_met": float(np.mean(lat < cadence_s * 1e3)),
            "subband_px_per_s": px / wall, "workspace_gb": used / 2 ** 30,
            "budget_gb": args.serve_budget_gb}


ROOFLINE_STAGES = ("ingest", "centre", "spread_peaks")
KERNEL_SOURCES = {"spread_peaks": ["paper_2103_15418_amd/csrc/filter.hip", "paper_2103_15418_amd/csrc/lpf_internal.h"],
                  "centre": ["paper_2103_15418_amd/csrc/filter.hip", "paper_2103_15418_amd/csrc/lpf_internal.h"],
                  "ingest": ["paper_2103_15418_amd/csrc/ingest.hip", "paper_2103_15418_amd/csrc/lpf_internal.h"]}
TRAFFIC_FILES = {"spread_peaks": "profiles/filter_strip_spread_instrument_16x1024.md",
                 "centre": "profiles/filter_strip_centre_instrument_16x1024.md",
                 "ingest": "profiles/ingest_instrument_16x1024.md"}


def sources_sha256(stage):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES.get(stage, []):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(stage):
    """HBM bytes per launch from the committed rocprofv3 counter summary of the
    stage's kernel (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known
    size), or None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_FILES.get(stage, ""))
    if stage not in TRAFFIC_FILES or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("sources_sha256") != sources_sha256(stage):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def network_batch(model_cls, wts, precision, n=1024, reps=10):
    """The network alone on n resident windows (events on its own stream)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    x = torch.randn((n, 16, 64), generator=g, device="cuda", dtype=torch.float32)
    m = model_cls(wts, precision=precision, max_batch=n)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        m.infer_windows(x, stream=s)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            m.infer_windows(x, stream=s)
        e1.record(s)
        s.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ach = CNN_FLOPS * n / (ms * 1e-3) / 1e12
    peak = FP32_MFMA_PEAK_TFLOPS if precision == 0 else BF16_MFMA_PEAK_TFLOPS
    return {"windows": n, "ms": ms, "achieved_tflops": ach, "peak_tflops": peak, "frac": ach / peak}


def paced_latency(ctx, model, frames, t_first, cadence_s):
    """Per-frame latency (completion of extract_flux minus arrival, host
    monotonic clock) with frames arriving every cadence_s: each frame is
    submitted at its arrival time and its completion is the moment an event
    recorded after its flux stage (on the context's stream) is seen done."""
    import torch
    lat = []
    pending = []
    t0 = time.perf_counter() + 0.01
    for k, cube in enumerate(frames):
        arrival = t0 + k * cadence_s
        while time.perf_counter() < arrival:
            pass
        ctx.ingest(t_first + k, cube)
        ctx.detect(want=False)
        ctx.extract_flux()
        ev = torch.cuda.Event()
        ev.record()
        pending.append(model.infer_async([ctx]))
        ev.synchronize()
        lat.append(time.perf_counter() - arrival)
        if len(pending) > 2:
            model.collect(pending.pop(0))
    while pending:
        model.collect(pending.pop(0))
    return np.array(lat) * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=52)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="instrument", choices=["instrument", "tiny"])
    ap.add_argument("--cpu-frames", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads generating cubes (and oracle processes in the CPU baseline)")
    ap.add_argument("--no-precision-forms", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--latency-frames", type=int, default=64)
    ap.add_argument("--latency-cadence-ms", type=float, default=5.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="real-time serving run (1 s cadence +- 100 ms); 600 reproduces the full scenario")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-pipeline", action="store_true",
                    help="ingest on the context's stream after the previous step's flux")
    ap.add_argument("--network-only", action="store_true",
                    help="only the network on 1024 resident windows per precision (counter runs)")
    ap.add_argument("--network-batch", type=int, default=1024, help="windows per call with --network-only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 1 GiB device-to-device once (reference for HBM counters)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_run(args.workload, args.cpu_frames, args.workers)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2103_15418_amd import Context, Model

    torch.cuda.set_device(0)
    if args.network_only:
        n = args.network_batch
        out = {name: network_batch(Model, synth.cnn_weights(), code, n=n) for code, name in ((0, "fp32"), (1, "bf16"),
                                                                                             (2, "fp16"))}
        print(json.dumps({f"network_batch{n}": out}), flush=True)
        return
    spec = _spec(args.workload)
    st = synth.Stream(spec)
    B, H, W = spec.B, spec.H, spec.W
    # untimed lead-in: the warmup steps, at least one monitoring window plus one
    # step (episodes end at t_last_det + 31), so that the network runs in the
    # timed steps; then the profiled pass and the timed steps, each on its own cube
    n_mon = 31
    lead = max(args.warmup, n_mon + 1 + 8)
    n_prof = max(4, min(args.warmup, 8))
    n_lat = 0 if args.no_latency else args.latency_frames
    n_total = lead + n_prof + args.steps + n_lat
    print(f"[bench] generating {n_total} cubes of {B}x{H}x{W}", file=sys.stderr, flush=True)
    pool = torch.empty((n_total, B, H, W), dtype=torch.float32, device="cuda")
    chunk = 16
    for c0 in range(0, n_total, chunk):
        fr = make_frames(st, range(c0, min(n_total, c0 + chunk)), args.workers)
        for i, f in enumerate(fr):
            pool[c0 + i].copy_(torch.from_numpy(f))
    del fr

    def run(precision, steps, frames=None, latency=False):
        """Lead-in, profiled pass, then `steps` timed steps.  Returns (elapsed s,
        host call times, stage profile, (dominant stage, its timed profile),
        windows inferred in the timed steps, config, latency array or None).
        frames: cubes to use instead of the device-resident pool (cycled)."""
        src = pool if frames is None else frames
        ctx = Context(B, H, W, sky_mask=st.mask, filter_precision=precision,
                      pipeline_ingest=0 if args.no_pipeline else 1)
        model = Model(synth.cnn_weights(), precision=precision, max_batch=1024)
        torch.cuda.synchronize()
        n_inf = [0]
        pending = []

        def step(t):
            # the network's results of step t are collected during step t + 2
            # (a pipelined context launches that network after the centre pass
            # of step t + 1), so the host enqueues the next frame while the
            # device finishes
            ctx.ingest(t, src[t % len(src)])
            ctx.detect(want=False)
            ctx.extract_flux()
            pending.append(model.infer_async([ctx]))
            if len(pending) > 2:
                mu, L, s_ = model.collect(pending.pop(0))
                n_inf[0] += len(mu)

        def drain():
            while pending:
                mu, L, s_ = model.collect(pending.pop(0))
                n_inf[0] += len(mu)

        for t in range(lead):
            step(t)
        drain()
        # untimed pass with events around every stage: stage times, dominant kernel
        ctx.profile(True)
        ctx.profile_read()
        for t in range(lead, lead + n_prof):
            step(t)
        drain()
        prof_all = ctx.profile_read()
        # dominant kernel among those with a throughput roofline (ingest: HBM; centre and
        # spread: matrix cores); QC, catalogue and flux are latency-bound one-workgroup or
        # few-workgroup kernels and are reported under "stages"
        dom = max((k for k in ROOFLINE_STAGES if prof_all.get(k, (0, 0))[1] > 0),
                  key=lambda k: prof_all[k][0] / prof_all[k][1])
        # timed run: events around the dominant kernel of every 8th step only (each
        # event pair costs the stream several microseconds)
        t_base = lead + n_prof
        n_inf[0] = 0
        host = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            f0 = time.perf_counter()
            if i % 8 == 0:
                ctx.profile(True, stages=[dom])
            elif i % 8 == 1:
                ctx.profile(False)
            step(t_base + i)
            host.append(time.perf_counter() - f0)
        drain()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof_timed = ctx.profile_read()
        ctx.profile(False)
        lat = None
        if latency and n_lat:
            lat = paced_latency(ctx, model, [src[t] for t in range(t_base + steps, t_base + steps + n_lat)],
                                t_base + steps, args.latency_cadence_ms * 1e-3)
        cfg = ctx.cfg
        del ctx, model
        return el, host, prof_all, (dom, prof_timed[dom]), n_inf[0], cfg, lat

    print(f"[bench] fp32: lead-in {lead} steps, timing {args.steps} steps", file=sys.stderr, flush=True)
    elapsed, host, prof, dom_timed, n_windows, cfg, lat = run(0, args.steps, latency=True)
    px_step = B * H * W
    value = args.steps * px_step / elapsed

    def stage_entry(name, ms, cnt):
        avg = ms / cnt
        ent = {"ms_total": round(ms, 4), "launches": cnt, "avg_ms": round(avg, 5)}
        if name == "ingest":
            ach = 24.0 * px_step / (avg * 1e-3) / 1e9
            ent.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS)
        elif name in ("centre", "spread_peaks"):
            # algorithmic work: two 1-D passes of 2k+1 taps (FMA = 2 FLOP) per pixel; both passes
            # run as banded products on the float32 matrix cores.  Algorithmic bytes: the centre
            # pass reads x and writes c and the signed residual plane (12 B per pixel), the
            # spread pass reads the residual plane (4 B per pixel; S is not stored).
            k = cfg.bg_halfwidth if cfg.bg_halfwidth > 0 else int(np.ceil(3 * cfg.bg_sigma))
            flops = 2.0 * 2 * (2 * k + 1) * px_step
            ach = flops / (avg * 1e-3) / 1e12
            bpp = 12.0 if name == "centre" else 4.0
            ent.update(bound="mfma", achieved=ach, peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=ach / FP32_MFMA_PEAK_TFLOPS,
                       hbm_view={"bytes_per_px": bpp, "achieved_gbs": bpp * px_step / (avg * 1e-3) / 1e9,
                                 "frac": bpp * px_step / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS})
        elif name == "network":
            # the network runs on the model's own stream, overlapped with the next step's
            # kernels: its event span is not a kernel duration (see network_batch1024)
            ent["note"] = "overlapped with the next step on the model stream"
        return ent

    # per-stage figures from the untimed pass with events around every stage
    stages = {name: stage_entry(name, ms, cnt) for name, (ms, cnt) in prof.items() if cnt > 0}
    # roofline of the dominant kernel from the events recorded around it in the timed steps
    dom, (dom_ms, dom_cnt) = dom_timed
    d = stage_entry(dom, dom_ms, dom_cnt)
    slowest = max((k for k in prof if k != "network" and prof[k][1] > 0), key=lambda k: prof[k][0] / prof[k][1])
    roof = {"kernel": dom, "bound": d.get("bound"), "achieved": d.get("achieved"),
            "peak": d.get("peak"), "unit": d.get("unit"), "frac": d.get("frac"),
            "traffic": stored_traffic(dom), "avg_ms": d["avg_ms"], "launches": dom_cnt,
            "note": "longest kernel with a throughput roof (ingest, centre, spread); longest stage "
                    f"overall in the profiled pass: {slowest}"}
    host_ms = np.array(host) * 1e3
    t_first = lead + n_prof
    stages_run = "QC + detect + associate + flux/backfill" + (" + network" if n_windows > 0 else "")
    out = {
        "metric": "subband-pixels/sec through detect+flux",
        "value": value,
        "unit": "subband-px/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        # the paper processes one 16 x 1024^2 cube in under 1 s (Titan RTX): >= 1.68e7 px/s
        "vs_baseline": value / (16 * 1024 * 1024 / 1.0) if args.workload == "instrument" else None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} subbands x {H}x{W}, "
                               f"{'circular sky mask, ' if spec.mask else ''}{spec.n_sources} dispersed sources, "
                               f"one distinct cube per step ({stages_run})",
                   "timed_steps_t": [t_first, t_first + args.steps - 1],
                   "lead_in_steps": lead,
                   "kappa": cfg.kappa, "bg_sigma": cfg.bg_sigma, "clip_iters": cfg.clip_iters,
                   "pipeline_ingest": int(cfg.pipeline_ingest),
                   "network_precision": "fp32", "windows_inferred": n_windows},
        "host_call_ms": {"p50": float(np.percentile(host_ms, 50)), "p99": float(np.percentile(host_ms, 99)),
                         "note": "host time of one step's calls in the timed run (enqueue, plus the "
                                 "collection of the network results of two steps earlier)"},
        "roofline": roof,
        "stages": stages,
        "stages_note": "per-stage event timings from an untimed pass (events around every stage); "
                       "the timed steps record events around the dominant kernel of every 8th step",
    }
    if lat is not None:
        out["latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "max": float(lat.max()), "frames": int(len(lat)),
                             "cadence_ms": args.latency_cadence_ms,
                             "definition": "completion of extract_flux (event on the context stream seen "
                                           "done by the host) minus the frame's arrival time; frames "
                                           "arrive at a fixed cadence after the timed steps"}
    # precision forms: bf16 / fp16 operands on MFMA (filters and network), float32 accumulation;
    # timed right after the float32 steps, under the same conditions
    if not args.no_precision_forms:
        forms = {}
        for code, name in ((1, "bf16"), (2, "fp16")):
            print(f"[bench] {name}: timing {args.steps} steps", file=sys.stderr, flush=True)
            el, hs, pr, _, nw, _, _ = run(code, args.steps)
            forms[name] = {"value": args.steps * px_step / el, "ms_per_step": el / args.steps * 1e3,
                           "stage_avg_ms": {k: round(v[0] / v[1], 5) for k, v in pr.items() if v[1]},
                           "windows_inferred": nw}
            forms[name]["error_vs_fp64"] = precision_errors(code, st, pool, Context, Model, synth)
        out["precision_forms"] = forms
    out["network_batch1024"] = {name: network_batch(Model, synth.cnn_weights(), code)
                                for code, name in ((0, "fp32"), (1, "bf16"), (2, "fp16"))}
    # the batch a step of the timed run hands over (about 30 ended episodes)
    out["network_batch32"] = {name: network_batch(Model, synth.cnn_weights(), code, n=32, reps=50)
                              for code, name in ((0, "fp32"), (1, "bf16"))}
    # cubes handed over from pinned host memory: the rate including the PCIe copy (not `value`)
    host_pool = [pool[t].cpu().pin_memory() for t in range(4)]
    n_h = min(args.steps, 20)
    el_h = run(0, n_h, frames=host_pool)[0]
    out["pcie_inclusive"] = {"value": n_h * px_step / el_h, "unit": "subband-px/s",
                             "ms_per_step": el_h / n_h * 1e3,
                             "note": "cubes copied host->device each step from pinned memory (4 cubes cycled)"}
    del host_pool
    if not args.no_serving:
        del pool
        torch.cuda.empty_cache()
        specs = synth.spec_serving_streams()
        masks = [synth.sky_mask(s.H, s.W) for s in specs]
        n_distinct = 3
        print(f"[bench] serving: generating {n_distinct} cubes for each of {len(specs)} streams",
              file=sys.stderr, flush=True)
        pools = []
        for s_ in specs:
            fr = make_frames(synth.Stream(s_), range(n_distinct), args.workers)
            pools.append([torch.from_numpy(f).cuda() for f in fr])
        del fr
        serve = {}
        print(f"[bench] serving: real time, {args.serve_seconds:.0f} s", file=sys.stderr, flush=True)
        serve["realtime_fp32"] = serving(args, 0, pools, specs, masks, args.serve_seconds, 1.0, 0.1)
        for code, name in ((0, "fp32"), (1, "bf16")):
            print(f"[bench] serving: {name} at 100x the cadence", file=sys.stderr, flush=True)
            serve[f"stress_{name}"] = serving(args, code, pools, specs, masks, 2.0, 0.01, 0.001, seed=1)
        out["serving"] = serve
        del pools
    if args.calibrate_copy:
        # plain device copy of known size (1 GiB, beyond the last-level cache), for scaling
        # the FETCH_SIZE / WRITE_SIZE counters of a profiled run
        src_ = torch.ones(256 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src_)
        torch.cuda.synchronize()
        dst.copy_(src_)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src_.numel() * 4
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline ({args.cpu_frames} oracle steps, child process)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
