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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=52)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="instrument", choices=["instrument", "tiny"])
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 256 MiB device-to-device once (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
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
    ctx = Context(B, H, W, sky_mask=st.mask)
    model = Model(synth.cnn_weights(), max_batch=1024)
    torch.cuda.synchronize()

    n_inferred = [0]

    def step(t):
        ctx.ingest(t, pool[t % n_pool])
        ctx.detect(want=False)
        ctx.extract_flux()
        mu, L, src = model.infer([ctx])
        n_inferred[0] += len(mu)

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    n_inferred[0] = 0
    lat = []
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        f0 = time.perf_counter()
        step(args.warmup + i)
        lat.append(time.perf_counter() - f0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)

    px_step = B * H * W
    value = args.steps * px_step / elapsed
    stages = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg = ms / cnt
        ent = {"ms_total": round(ms, 4), "launches": cnt, "avg_ms": round(avg, 5)}
        if name == "ingest":
            ach = 24.0 * px_step / (avg * 1e-3) / 1e9
            ent.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS)
        elif name in ("centre", "spread_peaks"):
            k = ctx.cfg.bg_halfwidth if ctx.cfg.bg_halfwidth > 0 else int(np.ceil(3 * ctx.cfg.bg_sigma))
            flops = 2.0 * 2 * (2 * k + 1) * px_step
            ach = flops / (avg * 1e-3) / 1e12
            ent.update(bound="alu", achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=ach / FP32_VECTOR_PEAK_TFLOPS)
        elif name == "network" and n_inferred[0] > 0:
            ach = CNN_FLOPS * n_inferred[0] / (ms * 1e-3) / 1e12
            ent.update(bound="mfma", achieved=ach, peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=ach / FP32_MFMA_PEAK_TFLOPS, windows=n_inferred[0])
        stages[name] = ent
    dom = max(stages, key=lambda s: stages[s]["ms_total"])
    d = stages[dom]
    roof = {"kernel": dom, "bound": d.get("bound"), "achieved": d.get("achieved"),
            "peak": d.get("peak"), "unit": d.get("unit"), "frac": d.get("frac"), "traffic": None}
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
                   "network_precision": "fp32", "windows_inferred": n_inferred[0]},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "roofline": roof,
        "stages": stages,
    }
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
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
