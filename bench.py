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
import collections
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


def timed_calls(fn, stream, steps, warmup, spin=True):
    """Runs fn() warmup+steps times on `stream` (after spin_up, unless the caller
    has just done it); returns per-call ms (HIP events)."""
    import torch
    if spin:
        spin_up(fn)
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


COPY_BYTES = 512 << 20
# The workloads the counter passes profile: the kernel whose dispatches are read,
# how many dispatches one call makes, and the launch shape pinned for it (under
# the counter profiler the tuner's timings are distorted and it would pick
# another; these are the shapes the timed runs use).
PROFILES = {
    "3d": {"kernel": "k_ecc_3d", "file": "k_ecc_3d_f32_512cubed", "per_call": 1,
           "what": "512^3 float32 GRF (seed 3), vertex filtration, 4096 bins over [min, max]",
           "shape": {"waves": 8, "wgs_per_cu": 3, "depth": 32}},
    "2d": {"kernel": "k_ecc_2d", "file": "k_ecc_2d_u16_16384sq", "per_call": 1,
           "what": "16384^2 uint16 GRF (seed 4, 4096 levels), vertex filtration, 4096 bins over [min, max]",
           "shape": {"waves": 4, "wgs_per_cu": 4, "depth": 256}},
    "batch": {"kernel": "k_ecc_batch", "file": "k_ecc_batch_u8_512images", "per_call": 1,
              "what": "the uneven 512-image uint8 batch (seed 5), vertex filtration, 256 bins, default batch shape",
              "shape": None},
    "c2": {"kernel": "k_ecc_3d<0, 0, false, false>", "file": "k_ecc_3d_u8_256cubed", "per_call": 1,
           "what": "256^3 uint8 smoothed noise (sigma 2, seed 2), vertex filtration, 256 bins over [0, 255]",
           "shape": {"waves": 4, "wgs_per_cu": 4, "depth": 16}},
    "minmax": {"kernel": "k_minmax", "file": "k_minmax_f32_512cubed", "per_call": 1,
               "what": "the AUTO-range min/max pass over the 512^3 float32 GRF (seed 3), 4096 bins",
               "shape": {"waves": 8, "wgs_per_cu": 3, "depth": 32}},
    "smooth": {"kernel": "k_smooth", "file": "k_smooth13_f32_8192sq", "per_call": 2,
               "what": "one 13-tap smoothing pass (rows, then columns) of an 8192^2 float32 GRF (seed 8)",
               "shape": None},
    "4d": {"kernel": "k_ecc_3d<2, 0, false, true>", "file": "k_ecc_3d_pair_f32_8x256cubed", "per_call": 1,
           "what": "the launch of the 7 pair terms (elementwise max of two neighbouring 256^3 hyperplanes, one "
                   "term per workgroup row of the grid) of one call on the 8 x 256^3 float32 GRF (seed 9), "
                   "vertex filtration, 4096 bins over [min, max]",
           "shape": None},
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", PROFILES["3d"]["file"] + "_traffic.txt")
TRAFFIC_SHAPE = PROFILES["3d"]["shape"]


def kernel_sources_sha256():
    """Hash of the sources the histogram kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_09087_amd", "csrc")
    for name in ("ecc_internal.h", "ecc_device.h", "ecc_kernels.hip", "ecc_batch.hip"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def spin_up(fn, seconds=0.15):
    """Calls fn back to back for `seconds` of wall time before a measurement: the
    device runs its first ~150 steps of the 512^3 workload up to 15% slower (its
    clocks ramp up under load, and drop again within half a second of idling)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    if time.perf_counter() - t0 >= seconds / 8:   # a long call is its own warm-up
        return
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def region_ms(fn, stream, steps, warmup):
    """Mean milliseconds per call of `steps` calls timed as one region: a HIP
    event before the first and one after the last (per-call events would add
    their own packets between the calls), after `warmup` untimed calls, with a
    synchronisation on both sides.  Also returns the region's wall time (s)."""
    import torch
    spin_up(fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t0


def traffic_bytes():
    """HBM bytes per launch of the histogram kernel on the 512^3 f32 step, from the
    committed rocprofv3 counter summary, if it was taken from the current kernel
    sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return int(fields["hbm_bytes_per_call"])
    except (KeyError, ValueError):
        return None


def profile_input(which):
    """(run, algorithmic bytes per call) for a profiled workload: run() makes one call."""
    import torch
    from paper_2203_09087_amd import ecc, synth
    dev = torch.device("cuda", 0)
    spec = PROFILES[which]
    ctx = ecc.Context(0, "vertex")
    if which == "smooth":
        a = synth.grf((8192, 8192), seed=8)
        t = torch.from_numpy(a).to(dev)
        o = torch.empty_like(t)
        taps = np.exp(-0.5 * (np.arange(13) - 6.0) ** 2 / 4.0)
        taps = (taps / taps.sum()).astype(np.float32)
        return ctx, (lambda: ctx.smooth13(t, taps, out=o)), 16 * int(a.size)
    if which == "batch":
        imgs = [torch.from_numpy(a).to(dev) for a in synth.batch_images(count=512, seed=5)]
        outs = [torch.empty(256, dtype=torch.int64, device=dev) for _ in imgs]
        return ctx, (lambda: ctx.compute_batch(imgs, 256, outs=outs)), int(sum(t.numel() for t in imgs))
    if which in ("3d", "minmax"):
        a = synth.grf((512, 512, 512), seed=3)
        rng = (float(a.min()), float(a.max())) if which == "3d" else "auto"
        t = torch.from_numpy(a).to(dev)
    elif which == "2d":
        a = synth.quantize_u16(synth.grf((16384, 16384), seed=4), 4096)
        rng = (int(a.min()), int(a.max()))
        t = torch.from_numpy(a.view(np.int16)).to(dev)
    elif which == "c2":
        a = synth.smoothed_noise_u8((256, 256, 256), sigma=2.0, seed=2)
        t = torch.from_numpy(a).to(dev)
        out = torch.empty(256, dtype=torch.int64, device=dev)
        ctx.set_launch_shape(t, 256, **spec["shape"])
        return ctx, (lambda: ctx.compute(t, 256, value_range=(0, 255), out=out)), int(a.nbytes)
    else:
        a = synth.grf((8, 256, 256, 256), seed=9)
        rng = (float(a.min()), float(a.max()))
        t = torch.from_numpy(a).to(dev)
    out = torch.empty(4096, dtype=torch.int64, device=dev)
    if spec["shape"]:
        ctx.set_launch_shape(t, 4096, **spec["shape"])
    return ctx, (lambda: ctx.compute(t, 4096, value_range=rng, out=out)), int(a.nbytes)


def traffic_run(which="3d"):
    """The program the counter passes profile: three plain copies of a 512 MiB
    buffer (the calibration kernel, known bytes) and three calls of a workload
    (PROFILES)."""
    import torch
    dev = torch.device("cuda", 0)
    ctx, run, alg = profile_input(which)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    log(f"profile run {which}: {alg} algorithmic bytes per call, shape {PROFILES[which]['shape']}")
    for _ in range(3):
        run()
    torch.cuda.synchronize()
    ctx.close()
    log("profile run done")


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, counter value summed over the dispatch's rows)}."""
    import csv
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, v = out.get(d, (r["Kernel_Name"], 0.0))
        out[d] = (name, v + float(r["Counter_Value"]))
    return out


def write_traffic(which, fetch_csv, write_csv):
    """Turns the FETCH_SIZE and WRITE_SIZE passes over traffic_run(which) into the
    profile summary (traffic_bytes() reads the 3D one).  Each counter is scaled by
    the bytes the 512 MiB calibration copy is known to move over what the counter
    reads for it (its three dispatches: the program's three largest copies)."""
    spec = PROFILES[which]
    n = spec["per_call"]
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")

    def calib(d):
        vals = sorted((v for name, v in d.values() if "copy" in name.lower()), reverse=True)[:3]
        if len(vals) < 3:
            raise SystemExit("calibration copies not found")
        return float(np.mean(vals))

    def calls(d):
        ids = sorted(k for k, (name, _) in d.items() if spec["kernel"] in name)[-3 * n:]
        if len(ids) < 3 * n:
            raise SystemExit(f"{spec['kernel']}: {len(ids)} dispatches, {3 * n} expected")
        return float(np.sum([d[k][1] for k in ids])) / 3.0
    copy_name = "__amd_rocclr_copyBuffer"
    cf, cw = calib(f), calib(w)
    fs, ws = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
    ef, ew = calls(f), calls(w)
    hf, hw = ef * 1024 * fs, ew * 1024 * ws
    alg = _alg_bytes(which)
    copy = (copy_name,)
    lines = [
        f"# HBM traffic per call of the histogram kernel ({spec['kernel']}, {n} dispatch(es) per call):",
        f"# {spec['what']}; counters in KiB per dispatch.",
        "# $REPO is the repository root, $OUT an output folder.",
        f"command_fetch: cd /tmp && timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv "
        f"-d $OUT/pmc_fetch_{which} -o run -- python3 $REPO/bench.py --traffic {which}",
        f"command_write: cd /tmp && timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv "
        f"-d $OUT/pmc_write_{which} -o run -- python3 $REPO/bench.py --traffic {which}",
        f"command_summary: python3 bench.py --write-traffic {which} FETCH_CSV WRITE_CSV",
        f"launch_shape: {spec['shape'] or 'default'}",
        f"calibration_kernel: {copy[0]} (the three largest copy dispatches)",
        f"calibration_bytes: {COPY_BYTES} read and {COPY_BYTES} written per dispatch",
        f"copy_fetch_kib: {cf:.1f}",
        f"copy_write_kib: {cw:.1f}",
        f"fetch_scale: {fs:.4f}",
        f"write_scale: {ws:.4f}",
        f"histogram_fetch_kib_per_call: {ef:.1f} (mean of the last 3 calls)",
        f"histogram_write_kib_per_call: {ew:.1f}",
        f"hbm_fetch_bytes_per_call: {int(round(hf))}",
        f"hbm_write_bytes_per_call: {int(round(hw))}",
        f"hbm_bytes_per_call: {int(round(hf + hw))}",
        f"algorithmic_bytes_per_call: {alg}",
        f"traffic_over_algorithmic: {(hf + hw) / alg:.3f}",
        f"kernel_sources_sha256: {kernel_sources_sha256()}",
    ]
    path = os.path.join(ROOT, "profiles", spec["file"] + "_traffic.txt")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _alg_bytes(which):
    """Algorithmic bytes of one call (each voxel read once)."""
    if which == "3d":
        return 512 ** 3 * 4
    if which == "2d":
        return 16384 ** 2 * 2
    if which == "minmax":
        return 512 ** 3 * 4
    if which == "smooth":
        return 16 * 8192 ** 2   # rows and columns each read and write every pixel
    if which == "c2":
        return 256 ** 3
    if which == "4d":
        return 7 * 2 * 256 ** 3 * 4   # each of the 7 pair terms reads two hyperplanes
    from paper_2203_09087_amd import synth
    return int(sum(int(np.prod(s)) for s in synth.batch_shapes(count=512, seed=5)))


TRACE_FILE = os.path.join(ROOT, "profiles", "k_ecc_3d_f32_512cubed_trace.md")
MAIN_KERNEL = "k_ecc_3d<2, 0, false, false>"


def write_trace_summary(db_path, bench_json):
    """Summarizes a `rocprofv3 --kernel-trace` database of `bench.py --no-side
    --no-serve --no-cpu` into the profiles folder: every kernel's statistics, and
    the histogram kernel's mean over the launches the benchmark timed with
    kernel events (the last `roofline.launches` dispatches: that pass's steps)
    beside the kernel time the benchmark measured itself."""
    import sqlite3
    res = json.loads([l for l in open(bench_json) if l.startswith("{")][-1])
    steps = int(res["steps"])
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    stats = {}
    for name, a, b in rows:
        stats.setdefault(name, []).append((b - a) / 1000.0)
    main = [(b - a) / 1000.0 for name, a, b in rows if MAIN_KERNEL in name]
    timed = main[-int(res["roofline"]["launches"]):]
    total = sum(sum(v) for v in stats.values())
    out = ["# Kernel trace: 512^3 float32 GRF step (bench.py defaults without side runs)", "",
           "Commands (on one MI355X, from /tmp, $REPO the repository root, $OUT an output folder):", "",
           f"    rocprofv3 --kernel-trace --stats -d $OUT/prof -o run -- python3 $REPO/bench.py "
           f"--steps {steps} --warmup {res['warmup']} --no-cpu --no-side --no-serve > $OUT/prof.json",
           "    python3 $REPO/bench.py --trace-summary $OUT/prof/run_results.db $OUT/prof.json", "",
           f"Histogram kernel `{MAIN_KERNEL}` over the {len(timed)} launches timed with kernel events "
           f"(launch shape {res.get('launch_shape')}): mean {np.mean(timed):.2f} us, "
           f"min {np.min(timed):.2f} us, max {np.max(timed):.2f} us.  The benchmark's own HIP-event "
           f"measurement in the same run: {res['roofline']['kernel_ms'] * 1000:.2f} us per launch "
           f"(roofline.kernel_ms); step {res['ms_per_step'] * 1000:.1f} us.  Earlier dispatches of the "
           "kernel are the launch-shape tuner's candidates and the passes timed without kernel events "
           "(each spun up to steady clocks first).", "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---:|---:|---:|---:|---:|"]
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        short = name.replace("ecc::(anonymous namespace)::", "")
        short = short if len(short) < 70 else short[:67] + "..."
        out.append(f"| `{short}` | {len(v)} | {np.mean(v):.2f} | {np.min(v):.2f} | {np.max(v):.2f} | "
                   f"{100 * sum(v) / total:.2f} |")
    with open(TRACE_FILE, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


SQ_A = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY "
        "SQ_ACTIVE_INST_VALU")
SQ_B = ("SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS SQ_INSTS_VMEM SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE "
        "SQ_WAIT_ANY SQ_ACTIVE_INST_MISC")


def write_sq_summary(which, csv_a, csv_b):
    """Summarizes two SQ counter passes over `bench.py --traffic which` (the last
    call's dispatches of the histogram kernel, at the pinned launch shape) into the
    profiles folder, with the issue and LDS figures derived from them."""
    spec = PROFILES[which]
    n = spec["per_call"]
    meta = {}
    import csv
    passes = []
    for path in (csv_a, csv_b):
        per = {}
        for r in csv.DictReader(open(path)):
            if spec["kernel"] not in r["Kernel_Name"]:
                continue
            key = (int(r["Dispatch_Id"]), r["Counter_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
            meta = {k: r[k] for k in ("Grid_Size", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size")}
        ids = sorted({d for d, _ in per})[-3 * n:]
        vals = {}
        for (d, c), v in per.items():
            if d in ids:
                vals[c] = vals.get(c, 0.0) + v
        # per call: the call's dispatches summed, the mean over the three calls
        passes.append({c: v / 3.0 for c, v in vals.items()})
    # a counter taken in both passes (GRBM_GUI_ACTIVE): the mean of the two
    m = collections.defaultdict(lambda: float("nan"))
    for c in set(passes[0]) | set(passes[1]):
        m[c] = float(np.mean([p[c] for p in passes if c in p]))
    simds, xcds, cus = 1024, 8, 256
    cyc = m["GRBM_GUI_ACTIVE"] / xcds
    slots = cyc / 4
    alg = _alg_bytes(which)
    esize = {"3d": 4, "2d": 2, "4d": 4, "batch": 1, "c2": 1, "minmax": 4, "smooth": 16}[which]
    kvox = alg / esize / 1000.0
    out = [f"# SQ counters: `{spec['kernel']}`, {spec['what']}", "",
           "Commands (one pass each, from /tmp, $REPO the repository root, $OUT an output folder):", "",
           f"    timeout -s KILL 120 rocprofv3 --pmc {SQ_A} --output-format csv -d $OUT/sqa_{which} "
           f"-o run -- python3 $REPO/bench.py --traffic {which}",
           f"    timeout -s KILL 120 rocprofv3 --pmc {SQ_B} --output-format csv -d $OUT/sqb_{which} "
           f"-o run -- python3 $REPO/bench.py --traffic {which}",
           f"    python3 $REPO/bench.py --sq-summary {which} $OUT/sqa_{which}/run_counter_collection.csv "
           f"$OUT/sqb_{which}/run_counter_collection.csv", "",
           f"Dispatch: grid {meta.get('Grid_Size')} work-items, workgroup {meta.get('Workgroup_Size')}, "
           f"LDS {meta.get('LDS_Block_Size')} B, scratch {meta.get('Scratch_Size')} B; launch shape "
           f"{spec['shape'] or 'default'}.  Values per call ({n} dispatch(es)), means over the last three calls.", "",
           "| counter | value |", "|---|---:|"]
    for c in sorted(m):
        out.append(f"| {c} | {m[c]:.4g} |")
    out += ["", "Derived (GRBM_GUI_ACTIVE summed over 8 XCDs; 1024 SIMDs, 256 CUs; a slot is one SIMD's",
            "four-cycle issue turn):", "",
            f"* kernel cycles per XCD: {cyc:.0f} ({cyc / 2.4e3:.1f} us at 2.4 GHz)",
            f"* instructions per slot per SIMD: VALU {m['SQ_INSTS_VALU'] / simds / slots:.2f}, "
            f"SALU {m['SQ_INSTS_SALU'] / simds / slots:.2f}, LDS {m['SQ_INSTS_LDS'] / simds / slots:.3f}",
            f"* VALU busy: {100 * 4 * m['SQ_ACTIVE_INST_VALU'] / (cyc * simds):.0f}% of SIMD cycles",
            f"* instructions per 1000 voxels: VALU {m['SQ_INSTS_VALU'] / kvox:.1f}, "
            f"SALU {m['SQ_INSTS_SALU'] / kvox:.1f}, LDS {m['SQ_INSTS_LDS'] / kvox:.2f}, "
            f"VMEM {m['SQ_INSTS_VMEM'] / kvox:.2f}",
            f"* LDS busy: {100 * m['SQ_LDS_IDX_ACTIVE'] / (cyc * cus):.0f}% of CU cycles, of which "
            f"{100 * m['SQ_LDS_BANK_CONFLICT'] / max(m['SQ_LDS_IDX_ACTIVE'], 1):.0f}% bank-conflict stalls",
            f"* mean resident waves per SIMD: {4 * m['SQ_WAVE_CYCLES'] / (cyc * simds):.2f}"]
    path = os.path.join(ROOT, "profiles", spec["file"] + "_sq.md")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


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
    # one thread on a smaller sample of the same field
    one = vol[:8]
    t1 = time.perf_counter()
    oracle.ecc(one, nbins, "vertex", value_range=(lo, hi), threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": round(sample.size / dt / 1e9, 4), "unit": "Gvoxels/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {planes} of {vol.shape[0]} planes of the 512^3 f32 field "
                      f"({sample.size} voxels, vertex filtration, {nbins} bins), {dt:.1f} s",
            "single_thread": {"value": round(one.size / dt1 / 1e9, 4), "sample": f"first 8 planes, {dt1:.2f} s"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pipeline_leg(ctx, stream, iters=1000):
    """The smoothing + ECC pipeline on a 1024^2 float32 GRF resident on the
    device: each iteration computes the ECC (1024 bins over the image's current
    [min, max]) and then smooths the image with 13 Gaussian taps (sigma 2)."""
    import torch
    from paper_2203_09087_amd import synth
    img = torch.from_numpy(synth.grf((1024, 1024), seed=8)).cuda()
    taps = np.exp(-0.5 * (np.arange(13) - 6.0) ** 2 / 4.0)
    taps = (taps / taps.sum()).astype(np.float32)
    out = torch.empty(1024, dtype=torch.int64, device=img.device)

    def one():
        ctx.compute(img, 1024, value_range="auto", out=out, stream=stream)
        ctx.smooth13(img, taps, out=img, stream=stream)

    def only_ecc():
        ctx.compute(img, 1024, value_range="auto", out=out, stream=stream)

    def only_smooth():
        ctx.smooth13(img, taps, out=img, stream=stream)

    m_one, wall = region_ms(one, stream, iters, 10)
    m_e, _ = region_ms(only_ecc, stream, 200, 5)
    m_s, _ = region_ms(only_smooth, stream, 200, 5)
    return {"image": [1024, 1024], "iterations": iters, "nbins": 1024, "range": "auto",
            "ms_per_iteration": round(m_one, 4), "ecc_ms": round(m_e, 4),
            "smooth_ms": round(m_s, 4), "wall_s": round(wall, 3)}


def fourd_leg(ctx, stream, nbins=4096):
    """A 4D image: an 8 x 256^3 float32 Gaussian random field (P(k) ~ k^-3 in four
    dimensions, seed 9), 4096 bins over its [min, max], vertex filtration."""
    import torch
    from paper_2203_09087_amd import synth
    shape = (8, 256, 256, 256)
    vol = synth.grf(shape, seed=9)
    lo, hi = float(vol.min()), float(vol.max())
    d = torch.from_numpy(vol).cuda()
    del vol
    out = torch.empty(nbins, dtype=torch.int64, device=d.device)
    shape_t = ctx.autotune(d, nbins, value_range=(lo, hi), reps=3, stream=stream)
    m, _ = region_ms(lambda: ctx.compute(d, nbins, value_range=(lo, hi), out=out, stream=stream), stream, 20, 3)
    # the same image as a batch of one: its passes share one persistent launch
    mb, _ = region_ms(lambda: ctx.compute_batch([d], nbins, value_ranges=[(lo, hi)], outs=[out], stream=stream),
                      stream, 20, 3)
    nv = int(np.prod(shape))
    gbs = nv * 4 / (m * 1e-3) / 1e9
    return {"shape": list(shape), "nbins": nbins, "ms": round(m, 3), "gvox_s": round(nv / (m * 1e-3) / 1e9, 2),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "passes": 2 * shape[0] - 1, "launch_shape": shape_t,
            "batched_ms": round(mb, 3), "batched_gvox_s": round(nv / (mb * 1e-3) / 1e9, 2),
            "batched_hbm_frac": round(nv * 4 / (mb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def streamed_large_leg(ctx, stream, n=2048):
    """A 2048^3 uint8 volume (8 GiB) in pinned host memory streamed in 256 MiB
    slabs (33 slab copies, the copies overlapping the counting), 256 bins; its
    result is checked against the same volume counted resident on the device.
    The volume tiles the 256^3 smoothed-noise block of C2 (sigma 2, seed 2)
    8 x 8 x 8 times."""
    import torch
    from paper_2203_09087_amd import synth
    log("streaming a 2048^3 u8 volume from pinned host memory ...")
    b = 256
    block = synth.smoothed_noise_u8((b, b, b), sigma=2.0, seed=2)
    host = torch.empty((n, n, n), dtype=torch.uint8, pin_memory=True)
    hv = host.numpy()
    for z in range(0, n, b):
        for y in range(0, n, b):
            for x in range(0, n, b):
                hv[z:z + b, y:y + b, x:x + b] = block
    del block
    out = torch.empty(256, dtype=torch.int64, device=stream.device)
    ms, _ = timed_calls(lambda: ctx.compute_streamed(host, 256, value_range=(0, 255), out=out, stream=stream),
                        stream, 3, 1)
    dev = host.to(stream.device)
    ref = ctx.compute(dev, 256, value_range=(0, 255), stream=stream)
    torch.cuda.synchronize()
    same = bool(torch.equal(out, ref))
    del dev, host
    m = float(np.mean(ms))
    nv = n ** 3
    return {"shape": [n, n, n], "dtype": "u8", "slab_planes": "auto (256 MiB)", "ms": round(m, 2),
            "gvox_s": round(nv / (m * 1e-3) / 1e9, 2), "host_to_device_gb_s": round(nv / (m * 1e-3) / 1e9, 1),
            "equals_device_resident_call": same}


def rotated_leg(ctx, stream, make, shape, copies, nbins, reps, warmup, label, batch_n=0):
    """One small workload timed call by call over `copies` device copies of the
    input (at least 1 GiB in all, more than the 256 MB Infinity Cache), each call
    on the next copy, so no call reads an input a recent call left in cache."""
    import torch
    img = make()
    one_d = torch.from_numpy(img).to(stream.device)
    pool = one_d.unsqueeze(0).expand((copies,) + tuple(img.shape)).contiguous()
    del one_d
    out = torch.empty(nbins, dtype=torch.int64, device=pool.device)
    shape_t = ctx.autotune(pool[0], nbins, reps=5, stream=stream)
    i = [0]

    def one():
        ctx.compute(pool[i[0] % copies], nbins, out=out, stream=stream)
        i[0] += 1
    ms, wall = timed_calls(one, stream, reps, warmup)
    # back to back without per-call events: the rate a stream of calls reaches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    per_call = (time.perf_counter() - t0) / reps * 1e3
    # the histogram kernel alone (HIP events around its launches): what the
    # device spends per image once the host's call overhead is out of the way
    ctx.set_kernel_timing(True)
    one()
    ctx.kernel_time()
    for _ in range(min(reps, 200)):
        one()
    k_ms, k_n = ctx.kernel_time()
    ctx.set_kernel_timing(False)
    k_avg = k_ms / max(1, k_n)
    batched = None
    if batch_n:
        # the same images as planned batches of batch_n distinct copies (tables
        # built once, so the host does not pace the launches), one launch each
        groups = [[pool[(g * batch_n + i) % copies] for i in range(batch_n)] for g in range(8)]
        bouts = [torch.empty(nbins, dtype=torch.int64, device=pool.device) for _ in range(batch_n)]
        plans = [ctx.plan_batch(g, nbins, outs=bouts) for g in groups]
        k = [0]

        def one_batch():
            plans[k[0] % len(plans)].launch(stream=stream)
            k[0] += 1
        mb, _ = region_ms(one_batch, stream, 40, 8)
        torch.cuda.synchronize()
        for pl in plans:
            pl.close()
        nvb = batch_n * int(np.prod(shape))
        batched = {"images_per_launch": batch_n, "how": "planned batches over the rotated copies", "ms": round(mb, 4), "images_per_s": round(batch_n / (mb * 1e-3), 1),
                   "gvox_s": round(nvb / (mb * 1e-3) / 1e9, 2),
                   "hbm_frac": round(nvb * img.itemsize / (mb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    nv = int(np.prod(shape))
    m = float(np.median(ms))
    res = {"workload": label, "shape": list(shape), "nbins": nbins, "calls": reps,
           "input_rotation": f"{copies} copies, {copies * img.nbytes / 2**30:.2f} GiB",
           "p10_ms": round(float(np.percentile(ms, 10)), 4), "p50_ms": round(m, 4),
           "p90_ms": round(float(np.percentile(ms, 90)), 4),
           "gvox_s": round(nv / (m * 1e-3) / 1e9, 2),
           "hbm_frac": round(nv * img.itemsize / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "back_to_back_ms_per_call": round(per_call, 4), "launch_shape": shape_t,
           "kernel_ms": round(k_avg, 4), "kernel_gvox_s": round(nv / (k_avg * 1e-3) / 1e9, 2),
           "kernel_hbm_frac": round(nv * img.itemsize / (k_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if batched:
        res["as_batches"] = batched
    del pool
    return res


def read_ceiling(vol_d, stream):
    """A measured streaming-read rate of the same 512 MiB: a read-only reduction
    (torch's max over the volume), best of 10."""
    import torch
    ms, _ = timed_calls(lambda: torch.amax(vol_d), stream, 10, 2)
    return vol_d.numel() * vol_d.element_size() / (min(ms) * 1e-3) / 1e9


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
    # untimed warm-up: first-use allocations and kernel loading, every lane, 2D and 3D
    warm = synth.serving_requests(float(max(rates)), 256, seed=7)
    wviews = [p2[q["offset"][0]:q["offset"][0] + q["shape"][0], q["offset"][1]:q["offset"][1] + q["shape"][1]]
              if len(q["shape"]) == 2 else
              p3[q["offset"][0]:q["offset"][0] + q["shape"][0], q["offset"][1]:q["offset"][1] + q["shape"][1],
                 q["offset"][2]:q["offset"][2] + q["shape"][2]] for q in warm]
    srv.run_open_loop([0.0] * len(wviews), lambda i: serve.Request(source=wviews[i], nbins=4096,
                                                                    value_range=(0, 4095)))
    srv.peak_held = 0
    srv.batches = 0
    del wviews
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
    # the same stream with an admission budget that binds: 256 MiB, against
    # requests of up to 113 MB (a 384^3 uint16 crop), at 2000 requests/s
    small = 256 << 20
    srv = serve.Server(budget_bytes=small, max_batch=64, lanes=2)
    srv.run_open_loop([0.0] * 64, lambda i: serve.Request(source=p2[:512, :512], nbins=4096, value_range=(0, 4095)))
    srv.peak_held = 0
    reqs = synth.serving_requests(2000.0, 4000, seed=6)
    views = []
    for q in reqs:
        o, sh = q["offset"], q["shape"]
        sl = tuple(slice(a, a + b) for a, b in zip(o, sh))
        views.append(p2[sl] if len(sh) == 2 else p3[sl])
    log("serving at 2000 req/s with a 256 MiB budget ...")
    t0 = time.perf_counter()
    done = srv.run_open_loop([q["t"] for q in reqs], lambda i: serve.Request(source=views[i], nbins=4096,
                                                                             value_range=(0, 4095)))
    wall = time.perf_counter() - t0
    summ = serve.latency_summary(done, wall)
    summ["budget_bytes"] = small
    summ["peak_held_bytes"] = srv.peak_held
    summ["largest_request_bytes"] = max(v.numel() * v.element_size() + 8 * 4096 for v in views)
    out["binding_budget_2000"] = summ
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
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--traffic", nargs="?", const="3d", choices=sorted(PROFILES),
                    help="only the program the counter passes profile (a workload of PROFILES)")
    ap.add_argument("--write-traffic", nargs=3, metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV"),
                    help="summarize the two counter passes into the profiles folder")
    ap.add_argument("--trace-summary", nargs=2, metavar=("RESULTS_DB", "BENCH_JSON"),
                    help="summarize a kernel-trace database into the profiles folder")
    ap.add_argument("--sq-summary", nargs=3, metavar=("WORKLOAD", "CSV_A", "CSV_B"),
                    help="summarize the two SQ counter passes into the profiles folder")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.trace_summary:
        write_trace_summary(*args.trace_summary)
        return
    if args.sq_summary:
        write_sq_summary(*args.sq_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the histogram of a multi-GPU "
                                   "run would be one all-reduce of nbins int64 (see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.traffic:
        traffic_run(args.traffic)
        return

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

    shape = None
    if not args.no_autotune:
        log("autotuning the launch shape ...")
        shape = ctx.autotune(vol_d, nbins, value_range=(lo, hi), reps=3, stream=stream)
    log("timing plain 512^3 ...")
    ms_mean, wall = region_ms(step, stream, args.steps, args.warmup)
    # per-step times for the percentiles: the same steps again, an event pair
    # around each (kept out of the region above, whose mean they would lengthen)
    ms, _ = timed_calls(step, stream, args.steps, 0)
    # The dominant kernel alone: the same steps again with HIP events recorded
    # around every launch of the histogram kernel on the call's stream (kept out
    # of the run above, whose step time they would lengthen).
    # Only the timed steps' launches carry the events (the spin-up calls run
    # without them, one synchronisation every 8 calls).
    spin_up(step)
    ctx.set_kernel_timing(True)
    ms_k, _ = timed_calls(step, stream, args.steps, 0, spin=False)
    k_ms, k_launches = ctx.kernel_time()
    ctx.set_kernel_timing(False)
    k_avg = k_ms / max(1, k_launches)
    nvox = vol.size
    gvox = nvox / (ms_mean * 1e-3) / 1e9
    alg_bytes = nvox * 4            # each f32 voxel read once
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    # a measured streaming rate beside the published peak: a device-to-device
    # copy of the same 512 MiB (bytes read plus bytes written), best of 10
    vol_copy = torch.empty_like(vol_d)
    ms_copy, _ = timed_calls(lambda: vol_copy.copy_(vol_d), stream, 10, 2)   # on the current stream
    copy_rate = 2 * alg_bytes / (min(ms_copy) * 1e-3) / 1e9
    del vol_copy

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
        "roofline": {"bound": "hbm", "kernel": "k_ecc_3d (f32, vertex)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_bytes(), "traffic_launch_shape": TRAFFIC_SHAPE,
                     "measured_copy_gb_s": round(copy_rate, 1),
                     "measured_copy_how": "device-to-device copy of the same 512 MiB, read + written bytes, best of 10",
                     "kernel_ms": round(k_avg, 4),
                     "launches": k_launches, "algorithmic_bytes": alg_bytes,
                     "step_ms_with_kernel_events": round(float(np.mean(ms_k)), 4)},
        "launch_shape": shape,
        "p10_ms": round(float(np.percentile(ms, 10)), 4),
        "p50_ms": round(float(np.percentile(ms, 50)), 4),
        "p90_ms": round(float(np.percentile(ms, 90)), 4),
        "p99_ms": round(float(np.percentile(ms, 99)), 4),
        "wall_s": round(wall, 3),
    }

    if not args.no_side:
        log("timing AUTO range ...")
        # AUTO and explicit calls alternate, so both see the same state of the
        # device; the min/max pass alone is the difference of their medians
        modes = []

        def alternate():
            auto = len(modes) % 2 == 0
            ctx.compute(vol_d, nbins, value_range="auto" if auto else (lo, hi), out=out, stream=stream)
            modes.append(auto)
        ms_ae, _ = timed_calls(alternate, stream, 40, 4)
        timed_modes = modes[-40:]   # the calls the 40 timings belong to
        ms_a = [m for m, a in zip(ms_ae, timed_modes) if a]
        ms_e = [m for m, a in zip(ms_ae, timed_modes) if not a]
        result["auto_range_ms"] = round(float(np.median(ms_a)), 4)
        mm_ms = max(1e-6, float(np.median(ms_a)) - float(np.median(ms_e)))
        mm_rate = alg_bytes / (mm_ms * 1e-3) / 1e9
        torch_rate = read_ceiling(vol_d, stream)
        result["roofline"]["minmax_pass_gb_s"] = round(mm_rate, 1)
        result["roofline"]["torch_amax_gb_s"] = round(torch_rate, 1)
        result["roofline"]["read_ceiling_gb_s"] = round(max(mm_rate, torch_rate), 1)
        result["roofline"]["read_ceiling_how"] = ("the faster of two read-only passes over the same 512 MiB: the "
                                                  "library's AUTO-range min/max pass (median AUTO step minus median "
                                                  "explicit step, the two alternating) and torch.amax (best of 10)")
        result["roofline"]["frac_of_read_ceiling"] = round(achieved / result["roofline"]["read_ceiling_gb_s"], 4)
        del vol_d
        log("generating 16384^2 u16 GRF ...")
        img2 = synth.quantize_u16(synth.grf((16384, 16384), seed=4), 4096)
        img2_d = torch.from_numpy(img2.view(np.int16)).to(dev)
        shape2 = None
        if not args.no_autotune:
            shape2 = ctx.autotune(img2_d, nbins, value_range="auto", reps=3, stream=stream)
        m2, _ = region_ms(lambda: ctx.compute(img2_d, nbins, value_range="auto", out=out,
                                              stream=stream), stream, 20, 3)
        lo2, hi2 = int(img2.min()), int(img2.max())
        m2e, _ = region_ms(lambda: ctx.compute(img2_d, nbins, value_range=(lo2, hi2), out=out,
                                               stream=stream), stream, 20, 3)
        result["plain_2d_u16"] = {"shape": [16384, 16384], "ms": round(m2, 4),
                                  "gvox_s": round(img2.size / (m2 * 1e-3) / 1e9, 2),
                                  "hbm_frac": round(img2.size * 2 / (m2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "range": "auto (a second read for the min/max pass)",
                                  "explicit_range_ms": round(m2e, 4),
                                  "explicit_range_gvox_s": round(img2.size / (m2e * 1e-3) / 1e9, 2),
                                  "explicit_range_hbm_frac": round(img2.size * 2 / (m2e * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "launch_shape": shape2}
        del img2_d, img2

        log("small configs (inputs rotated over 1 GiB) ...")
        result["small_2d_u8"] = rotated_leg(ctx, stream, lambda: synth.uniform_u8((256, 256), seed=1), (256, 256),
                                            16384, 256, 1000, 20, "256^2 uint8 uniform noise (seed 1), 256 bins",
                                            batch_n=1024)
        result["small_3d_u8"] = rotated_leg(ctx, stream,
                                            lambda: synth.smoothed_noise_u8((256, 256, 256), sigma=2.0, seed=2),
                                            (256, 256, 256), 64, 256, 200, 10,
                                            "256^3 uint8 smoothed noise (sigma 2, seed 2), 256 bins")
        log("generating the uneven batch ...")
        imgs = synth.batch_images(count=512, seed=5)
        nv = int(sum(a.size for a in imgs))
        dev_imgs = [torch.from_numpy(a).to(dev) for a in imgs]
        outs = [torch.empty(256, dtype=torch.int64, device=dev) for _ in imgs]
        mb, _ = region_ms(lambda: ctx.compute_batch(dev_imgs, 256, outs=outs, stream=stream), stream, 5, 2)

        def per_image():
            for a, o in zip(dev_imgs, outs):
                ctx.compute(a, 256, out=o, stream=stream)
        mp, _ = region_ms(per_image, stream, 5, 2)
        # the same batch planned once, its launch shape tuned, and replayed from a
        # captured HIP graph
        plan = ctx.plan_batch(dev_imgs, 256, outs=outs)
        plan_shape = plan.autotune(reps=3, stream=stream)
        ml, _ = region_ms(lambda: plan.launch(stream=stream), stream, 5, 2)
        gs = torch.cuda.Stream(dev)
        gs.wait_stream(stream)
        with torch.cuda.stream(gs):
            plan.launch(stream=gs)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            plan.launch(stream=gs)
        mg, _ = region_ms(graph.replay, stream, 5, 2)
        torch.cuda.synchronize()
        plan.close()
        result["batched"] = {"images": len(imgs), "voxels": nv, "ms": round(mb, 3),
                             "images_per_s": round(len(imgs) / (mb * 1e-3), 1),
                             "gvox_s": round(nv / (mb * 1e-3) / 1e9, 2),
                             "hbm_frac": round(nv / (mb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "planned_ms": round(ml, 3), "plan_shape": plan_shape,
                             "graph_replay_ms": round(mg, 3),
                             "per_image_calls_ms": round(mp, 3),
                             "speedup_vs_per_image": round(mp / mb, 3)}
        del dev_imgs, outs

    if not args.no_side:
        log("streaming the 512^3 f32 field from pinned host memory ...")
        host = torch.from_numpy(vol).pin_memory()
        ms_s, _ = timed_calls(lambda: ctx.compute_streamed(host, nbins, value_range=(lo, hi), out=out,
                                                           stream=stream), stream, 5, 1)
        msv = float(np.mean(ms_s))
        result["streamed_from_host"] = {"shape": [512, 512, 512], "slab_planes": "auto (256 MiB)",
                                        "ms": round(msv, 3), "gvox_s": round(nvox / (msv * 1e-3) / 1e9, 2),
                                        "host_to_device_gb_s": round(nvox * 4 / (msv * 1e-3) / 1e9, 1)}
        del host
        result["streamed_large"] = streamed_large_leg(ctx, stream)

    if not args.no_side:
        result["pipeline"] = pipeline_leg(ctx, stream)
        log("4D image ...")
        result["fourd"] = fourd_leg(ctx, stream)

    if not args.no_side and not args.no_serve:
        result["serving"] = serving_leg(dev)

    if not args.no_cpu:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(vol, nbins, lo, hi)

    result["configs"] = config_summary(result)
    print(json.dumps(result), flush=True)


def config_summary(r):
    """Gvoxels/s and fraction of HBM peak of each of the five workloads, gathered
    from the legs above (None where a leg was skipped)."""
    def pick(d, *keys):
        return {k: d.get(k) for k in keys} if d else None
    c = {"C1 256^2 u8 uniform, 256 bins": pick(r.get("small_2d_u8"), "p50_ms", "gvox_s", "hbm_frac", "kernel_ms",
                                                "kernel_gvox_s", "kernel_hbm_frac", "as_batches"),
         "C2 256^3 u8 smoothed, 256 bins": pick(r.get("small_3d_u8"), "p50_ms", "gvox_s", "hbm_frac", "kernel_ms",
                                                "kernel_gvox_s", "kernel_hbm_frac"),
         "C3 512^3 f32 GRF, 4096 bins, explicit range": {"ms": r.get("ms_per_step"), "gvox_s": r.get("value"),
                                                         "kernel_hbm_frac": r["roofline"]["frac"]},
         "C3 16384^2 u16 GRF, 4096 bins": pick(r.get("plain_2d_u16"), "ms", "gvox_s", "hbm_frac", "explicit_range_ms",
                                               "explicit_range_gvox_s", "explicit_range_hbm_frac"),
         "C4 512-image batch, 256 bins": pick(r.get("batched"), "ms", "planned_ms", "gvox_s", "hbm_frac",
                                              "speedup_vs_per_image")}
    srv = r.get("serving")
    c["C5 serving, 4096 bins"] = ({rate: pick(v, "p50_ms", "p99_ms", "completed_per_s", "gvox_s")
                                   for rate, v in srv["rates"].items()} if srv else None)
    if srv and "binding_budget_2000" in srv:
        c["C5 serving, 4096 bins"]["2000 with a 256 MiB budget"] = pick(srv["binding_budget_2000"], "p50_ms",
                                                                        "p99_ms", "completed_per_s",
                                                                        "peak_held_bytes")
    return c


if __name__ == "__main__":
    main()
