#!/usr/bin/env python3
"""Throughput of the transient-detection hot path on one MI355X.

One step = one synthetic image cube of the instrument workload (16 subbands
x 1024 x 1024 in a circular sky mask, 50 dispersed point sources, N(0,1)
noise on a smooth background) taken through every stage: quality control +
image cache, centre/spread filters + threshold + peaks, association, flux +
backward fill, and the network on the episodes that end at that step.
Cubes are generated up front and resident in HBM before timing starts.

Prints one JSON line: subband-pixels per second (metric of the paper's
real-time claim: a 16 x 1024^2 cube per 1 s step), per-step latency
percentiles, the roofline of the dominant kernel (timed with HIP events
recorded by the library on its stream) and the FP64 oracle's rate on a
bounded sample of the same workload on the host CPU.
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
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


def _gen_frame(args):
    spec_name, t = args
    import synth
    spec = synth.spec_instrument() if spec_name == "instrument" else synth.spec_tiny()
    return t, synth.Stream(spec).frame(t)


def make_frames(spec_name, n, workers):
    if workers <= 1:
        return [(_gen_frame((spec_name, t))[1]) for t in range(n)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        out = dict(pool.imap_unordered(_gen_frame, [(spec_name, t) for t in range(n)]))
    return [out[t] for t in range(n)]


def cpu_baseline(spec_name, n_frames):
    """FP64 oracle, single process, on the first n_frames steps of the workload."""
    import synth
    from oracle.config import OracleConfig
    from oracle.pipeline import OracleStream
    spec = synth.spec_instrument() if spec_name == "instrument" else synth.spec_tiny()
    st = synth.Stream(spec)
    orc = OracleStream(OracleConfig(B=spec.B, H=spec.H, W=spec.W, sky_mask=st.mask,
                                    freqs_mhz=st.freqs))
    frames = [st.frame(t) for t in range(n_frames)]
    t0 = time.perf_counter()
    for t, f in enumerate(frames):
        orc.ingest(t, f)
        orc.detect()
        orc.extract_flux()
    dt = time.perf_counter() - t0
    px = n_frames * spec.B * spec.H * spec.W
    return {"value": px / dt, "unit": "subband-px/s", "cores": 1, "kind": "oracle",
            "sample": f"steps 0-{n_frames - 1} of the {spec_name} workload "
                      f"({spec.B}x{spec.H}x{spec.W}): ingest+detect+extract_flux, "
                      f"numpy float64, one process, {dt:.1f} s"}


def precision_errors(code, st, pool, Context, Model, synth):
    """Max / median error relative to the FP64 oracle's condition scale: C and S
    on band 0 of step 0, network outputs on 32 seeded windows."""
    import torch
    from oracle import cnn as ocnn
    from oracle.filters import centre_spread, correlate_2d, taps_1d
    spec = st.spec
    c = Context(spec.B, spec.H, spec.W, sky_mask=st.mask, filter_precision=code, debug_planes=1)
    c.ingest(0, pool[0])
    c.detect(want=False)
    Cd, Sd = c.debug_read("centre")[0], c.debug_read("spread")[0]
    del c
    X = pool[0, 0].cpu().numpy()
    M = st.mask.astype(bool)
    g = taps_1d(0, 8.0, 24)
    C, S, den = centre_spread(X, M, g)
    pos = (den > 0) & M
    safe = np.where(den > 0, den, 1.0)
    scC = correlate_2d(M * np.abs(X.astype(np.float64)), g) / safe
    scS = correlate_2d(M * (np.abs(X.astype(np.float64)) + np.abs(C)) ** 2, g) / safe
    eC = (np.abs(Cd - C) / np.maximum(scC, 1e-30))[pos]
    eS = (np.abs(Sd - S) / np.maximum(scS, 1e-30))[pos]
    wts = synth.cnn_weights()
    x = (np.random.default_rng(0).standard_normal((32, 16, 64)) * 2.0).astype(np.float32)
    m = Model(wts, precision=code, max_batch=32)
    mu, L = m.infer_windows(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    raw = ocnn.forward_raw(x.astype(np.float64), wts)
    mo, Lo = ocnn.head(raw)
    a = x.astype(np.float64)[:, None]
    for l in range(1, 5):
        a = ocnn.act(ocnn.conv3x3(a, wts[f"conv{l}.w"], wts[f"conv{l}.b"]), wts["alpha"])
    h = ocnn.act(a.reshape(len(x), -1) @ wts["fc1.w"].astype(np.float64).T + wts["fc1.b"], wts["alpha"])
    sc = np.abs(h) @ np.abs(wts["fc2.w"].astype(np.float64)).T + np.abs(wts["fc2.b"])
    en = np.concatenate([np.abs(mu.cpu().numpy() - mo) / sc[:, :4], np.abs(L.cpu().numpy() - Lo) / sc[:, 4:]], 1)
    return {"scale": "|error| / condition scale (filters: G*(M|x|) and G*(M(|x|+|c|)^2) over G*M; "
                     "network: |W_fc2||h| + |b_fc2| with exact hidden activations h)",
            "centre": [float(eC.max()), float(np.median(eC))],
            "spread": [float(eS.max()), float(np.median(eS))],
            "network_mu": [float(en[:, :4].max()), float(np.median(en[:, :4]))],
            "network_L": [float(en[:, 4:].max()), float(np.median(en[:, 4:]))]}


def _gen_serving_frame(args):
    k, t = args
    import synth
    spec = synth.spec_serving_streams()[k]
    return (k, t), synth.Stream(spec).frame(t)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=52)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="instrument", choices=["instrument", "tiny"])
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-precision-forms", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="real-time serving run (1 s cadence +- 100 ms); 600 reproduces the full scenario")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-pipeline", action="store_true",
                    help="ingest on the context's stream after the previous step's flux")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 1 GiB device-to-device once (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2103_15418_amd import Context, Model

    torch.cuda.set_device(0)
    spec = synth.spec_instrument() if args.workload == "instrument" else synth.spec_tiny()
    st = synth.Stream(spec)
    B, H, W = spec.B, spec.H, spec.W
    n_pool = min(spec.T, args.warmup + args.steps)
    print(f"[bench] generating {n_pool} cubes of {B}x{H}x{W}", file=sys.stderr, flush=True)
    frames = make_frames(args.workload, n_pool, args.workers)
    pool = torch.empty((n_pool, B, H, W), dtype=torch.float32, device="cuda")
    for i, f in enumerate(frames):
        pool[i].copy_(torch.from_numpy(f))
    del frames
    def run(precision, steps, warmup, frames=None):
        """Times `steps` steps after `warmup`; returns (elapsed s, latencies, stage profile, windows).
        frames: the cubes to cycle through (default: the device-resident pool)."""
        frames = pool if frames is None else frames
        # the next step's ingest and QC run beside this step's catalogue and flux
        # (the cubes are resident before the loop starts)
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
            ctx.ingest(t, frames[t % len(frames)])
            ctx.detect(want=False)
            ctx.extract_flux()
            pending.append(model.infer_async([ctx]))
            if len(pending) > 2:
                mu, L, src = model.collect(pending.pop(0))
                n_inf[0] += len(mu)

        def drain():
            while pending:
                mu, L, src = model.collect(pending.pop(0))
                n_inf[0] += len(mu)

        for t in range(warmup):
            step(t)
        drain()
        # untimed pass with events around every stage: stage times, dominant kernel
        n_prof = max(4, min(warmup, 8))
        ctx.profile(True)
        ctx.profile_read()
        for t in range(warmup, warmup + n_prof):
            step(t)
        drain()
        prof_all = ctx.profile_read()
        dom = max((k for k in prof_all if k != "network" and prof_all[k][1] > 0),
                  key=lambda k: prof_all[k][0] / prof_all[k][1])
        # timed run: events around the dominant kernel of every 8th step only (each
        # event pair costs the stream several microseconds)
        t_base = warmup + n_prof
        n_inf[0] = 0
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            f0 = time.perf_counter()
            if i % 8 == 0:
                ctx.profile(True, stages=[dom])
            elif i % 8 == 1:
                ctx.profile(False)
            step(t_base + i)
            lat.append(time.perf_counter() - f0)
        drain()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof_timed = ctx.profile_read()
        ctx.profile(False)
        cfg = ctx.cfg
        del ctx, model
        return el, lat, prof_all, (dom, prof_timed[dom]), n_inf[0], cfg

    print(f"[bench] fp32: warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr, flush=True)
    elapsed, lat, prof, dom_timed, n_windows, cfg = run(0, args.steps, args.warmup)
    n_inferred = [n_windows]

    class _C:  # configuration of the timed run, for the stage rooflines
        pass
    ctx = _C()
    ctx.cfg = cfg
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
            k = ctx.cfg.bg_halfwidth if ctx.cfg.bg_halfwidth > 0 else int(np.ceil(3 * ctx.cfg.bg_sigma))
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
    roof = {"kernel": dom, "bound": d.get("bound"), "achieved": d.get("achieved"),
            "peak": d.get("peak"), "unit": d.get("unit"), "frac": d.get("frac"),
            "traffic": stored_traffic(dom), "avg_ms": d["avg_ms"], "launches": dom_cnt}
    lat_ms = np.array(lat) * 1e3
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
                               f"one cube per step (QC + detect + associate + flux/backfill + network)",
                   "kappa": ctx.cfg.kappa, "bg_sigma": ctx.cfg.bg_sigma, "clip_iters": ctx.cfg.clip_iters,
                   "pipeline_ingest": int(ctx.cfg.pipeline_ingest),
                   "network_precision": "fp32", "windows_inferred": n_inferred[0]},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "roofline": roof,
        "stages": stages,
        "stages_note": "per-stage event timings from an untimed pass (events around every stage); "
                       "the timed steps record events around the dominant kernel of every 8th step",
    }
    out["network_batch1024"] = {name: network_batch(Model, synth.cnn_weights(), code)
                                for code, name in ((0, "fp32"), (1, "bf16"), (2, "fp16"))}
    # cubes handed over from pinned host memory: the rate including the PCIe copy (not `value`)
    host_pool = [f.cpu().pin_memory() for f in pool[:2]]
    el_h, _, _, _, _, _ = run(0, min(args.steps, 20), 2, frames=host_pool)
    out["pcie_inclusive"] = {"value": min(args.steps, 20) * px_step / el_h, "unit": "subband-px/s",
                             "ms_per_step": el_h / min(args.steps, 20) * 1e3,
                             "note": "cubes copied host->device each step from pinned memory"}
    del host_pool
    # precision forms: bf16 / fp16 operands on MFMA (filters and network), float32 accumulation
    if not args.no_precision_forms:
        forms = {}
        for code, name in ((1, "bf16"), (2, "fp16")):
            print(f"[bench] {name}: timing {args.steps} steps", file=sys.stderr, flush=True)
            el, lt, pr, _, nw, _ = run(code, args.steps, args.warmup)
            forms[name] = {"value": args.steps * px_step / el, "ms_per_step": el / args.steps * 1e3,
                           "p99_ms": float(np.percentile(np.array(lt) * 1e3, 99)),
                           "stage_avg_ms": {k: round(v[0] / v[1], 5) for k, v in pr.items() if v[1]},
                           "windows_inferred": nw}
            forms[name]["error_vs_fp64"] = precision_errors(code, st, pool, Context, Model, synth)
        out["precision_forms"] = forms
    if not args.no_serving:
        del pool
        torch.cuda.empty_cache()
        specs = synth.spec_serving_streams()
        masks = [synth.sky_mask(s.H, s.W) for s in specs]
        n_distinct = 3
        print(f"[bench] serving: generating {n_distinct} cubes for each of {len(specs)} streams",
              file=sys.stderr, flush=True)
        jobs = [(k, t) for k in range(len(specs)) for t in range(n_distinct)]
        if args.workers > 1:
            with mp.get_context("fork").Pool(args.workers) as gp:
                gen = dict(gp.imap_unordered(_gen_serving_frame, jobs))
        else:
            gen = dict(_gen_serving_frame(j) for j in jobs)
        pools = [[torch.from_numpy(gen[(k, t)]).cuda() for t in range(n_distinct)] for k in range(len(specs))]
        del gen
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
        src = torch.ones(256 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline ({args.cpu_frames} oracle steps)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_frames)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
