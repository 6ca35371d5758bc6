"""Benchmark of the ECC hot path on one MI355X.

A step is one full pass of the plain path (bin -> per-voxel Euler contribution
-> LDS histogram -> merge -> prefix scan) over the 512^3 float32 Gaussian random
field (power spectrum k^-3) with 4096 bins over [min, max], the input already
resident in HBM.  The JSON line reports throughput in Gvoxels/s, the roofline of
the dominant kernel against MI355X HBM bandwidth, side measurements (the 16384^2
uint16 field, the uneven 512-image batch against per-image calls), and the CPU
oracle on a bounded sample of the same volume.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-side]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_calls(fn, stream, steps, warmup):
    """Runs fn() warmup+steps times on `stream`; returns per-call ms (HIP events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [s.elapsed_time(e) for s, e in zip(starts, ends)], wall


def cpu_baseline(vol, nbins, lo, hi, target_s=12.0):
    """The oracle as it is, on the first planes of the volume (bounded sample)."""
    import oracle
    oracle.build(force=False)
    threads = max(1, min(os.cpu_count() or 1, 16))
    planes = 4
    t0 = time.perf_counter()
    oracle.ecc(vol[:planes], nbins, "vertex", value_range=(lo, hi), threads=threads)
    dt = time.perf_counter() - t0
    per_plane = max(dt / planes, 1e-4)
    planes = int(min(vol.shape[0], max(planes, target_s / per_plane)))
    sample = vol[:planes]
    t0 = time.perf_counter()
    oracle.ecc(sample, nbins, "vertex", value_range=(lo, hi), threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample.size / dt / 1e9, 4), "unit": "Gvoxels/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {planes} of {vol.shape[0]} planes of the 512^3 f32 field "
                      f"({sample.size} voxels, vertex filtration, {nbins} bins), {dt:.1f} s"}


def serving_leg(dev, rates=(100, 200, 500, 1000, 2000, 5000), seconds=2.0, max_requests=4000):
    """Open-loop Poisson request streams over crops of two GRF pools (uint16,
    4096 levels), 4096 bins, HBM-footprint admission; p50/p99 per rate."""
    import torch
    from paper_2203_09087_amd import serve, synth
    log("generating serving pools ...")
    p2 = torch.from_numpy(synth.quantize_u16(synth.grf((4096, 4096), seed=61), 4096).view(np.int16)).to(dev)
    p3 = torch.from_numpy(synth.quantize_u16(synth.grf((384, 384, 384), seed=62), 4096).view(np.int16)).to(dev)
    torch.cuda.synchronize()
    budget = 8 << 30
    out = {"budget_bytes": budget, "max_batch": 64, "lanes": 2, "nbins": 4096, "rates": {}}
    srv = serve.Server(budget_bytes=budget, max_batch=64, lanes=2)
    for rate in rates:
        n = int(min(max_requests, max(200, rate * seconds)))
        reqs = synth.serving_requests(float(rate), n, seed=6)
        views = []
        for q in reqs:
            o, s = q["offset"], q["shape"]
            if len(s) == 2:
                views.append(p2[o[0]:o[0] + s[0], o[1]:o[1] + s[1]])
            else:
                views.append(p3[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]])
        arrivals = [q["t"] for q in reqs]
        log(f"serving at {rate} req/s, {n} requests ...")
        t0 = time.perf_counter()
        done = srv.run_open_loop(arrivals, lambda i: serve.Request(source=views[i], nbins=4096,
                                                                   value_range=(0, 4095)))
        wall = time.perf_counter() - t0
        summ = serve.latency_summary(done, wall)
        summ["gvox_s"] = round(sum(v.numel() for v in views) / wall / 1e9, 2)
        summ["peak_held_bytes"] = srv.peak_held
        out["rates"][str(rate)] = summ
    out["batches"] = srv.batches
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the histogram of a multi-GPU "
                                   "run would be one all-reduce of nbins int64 (see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2203_09087_amd import ecc, synth

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    nbins = 4096

    log("generating 512^3 f32 GRF ...")
    vol = synth.grf((512, 512, 512), seed=3)
    lo, hi = float(vol.min()), float(vol.max())
    vol_d = torch.from_numpy(vol).to(dev)
    ctx = ecc.Context(0, "vertex")
    out = torch.empty(nbins, dtype=torch.int64, device=dev)

    def step():
        ctx.compute(vol_d, nbins, value_range=(lo, hi), out=out, stream=stream)

    log("timing plain 512^3 ...")
    ms, wall = timed_calls(step, stream, args.steps, args.warmup)
    ms_mean = float(np.mean(ms))
    nvox = vol.size
    gvox = nvox / (ms_mean * 1e-3) / 1e9
    alg_bytes = nvox * 4
    achieved = alg_bytes / (ms_mean * 1e-3) / 1e9

    result = {
        "metric": "Gvoxels/s (plain single-image ECC, 512^3 f32, 4096 bins)",
        "value": round(gvox, 2),
        "unit": "Gvoxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_mean, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 float32 Gaussian random field (P(k)~k^-3, seed 3), "
                               "4096 bins over [min,max], vertex filtration, one ECC per step",
                   "shape": [512, 512, 512], "nbins": nbins, "range": "explicit"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "p50_ms": round(float(np.percentile(ms, 50)), 4),
        "p99_ms": round(float(np.percentile(ms, 99)), 4),
        "wall_s": round(wall, 3),
    }

    if not args.no_side:
        log("timing AUTO range ...")
        ms_a, _ = timed_calls(lambda: ctx.compute(vol_d, nbins, value_range="auto", out=out,
                                                  stream=stream), stream, 20, 3)
        result["auto_range_ms"] = round(float(np.mean(ms_a)), 4)
        del vol_d
        log("generating 16384^2 u16 GRF ...")
        img2 = synth.quantize_u16(synth.grf((16384, 16384), seed=4), 4096)
        img2_d = torch.from_numpy(img2.view(np.int16)).to(dev)
        ms2, _ = timed_calls(lambda: ctx.compute(img2_d, nbins, value_range="auto", out=out,
                                                 stream=stream), stream, 20, 3)
        m2 = float(np.mean(ms2))
        result["plain_2d_u16"] = {"shape": [16384, 16384], "ms": round(m2, 4),
                                  "gvox_s": round(img2.size / (m2 * 1e-3) / 1e9, 2),
                                  "hbm_frac": round(img2.size * 2 / (m2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del img2_d, img2

        log("generating the uneven batch ...")
        imgs = synth.batch_images(count=512, seed=5)
        nv = int(sum(a.size for a in imgs))
        dev_imgs = [torch.from_numpy(a).to(dev) for a in imgs]
        outs = [torch.empty(256, dtype=torch.int64, device=dev) for _ in imgs]
        ms_b, _ = timed_calls(lambda: ctx.compute_batch(dev_imgs, 256, outs=outs, stream=stream),
                              stream, 5, 2)

        def per_image():
            for a, o in zip(dev_imgs, outs):
                ctx.compute(a, 256, out=o, stream=stream)
        ms_p, _ = timed_calls(per_image, stream, 5, 2)
        mb, mp = float(np.mean(ms_b)), float(np.mean(ms_p))
        result["batched"] = {"images": len(imgs), "voxels": nv, "ms": round(mb, 3),
                             "images_per_s": round(len(imgs) / (mb * 1e-3), 1),
                             "gvox_s": round(nv / (mb * 1e-3) / 1e9, 2),
                             "per_image_calls_ms": round(mp, 3),
                             "speedup_vs_per_image": round(mp / mb, 3)}
        del dev_imgs, outs

    if not args.no_side and not args.no_serve:
        result["serving"] = serving_leg(dev)

    if not args.no_cpu:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(vol, nbins, lo, hi)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
