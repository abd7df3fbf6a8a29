"""Benchmark: Shack-Hartmann frames/s for 6 LGS sensors of 80x80 sub-apertures on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--frames-per-step B]

A step is one sh_wfs_measure launch over B frames of the 39 m workload
(6 LGS x 4928 valid 10x10-px sub-apertures, FFT 40, sodium kernel,
16x16 detector, 500 photons + 3 e- read noise, thresholded centroid).
OPD frames are resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# nominal FFT flops of one 40x40 complex 2-D transform: 5 N^2 log2(N^2); three per sub-aperture
FLOP_PER_SUBAP = 3 * 5 * 40 * 40 * math.log2(40 * 40)
PEAK_FP32_TFLOPS = 157.3
CSRC = os.path.join(ROOT, "paper_1408_0698_amd", "csrc")
TRAFFIC = os.path.join(ROOT, "profiles", "wfs_fused_lgs39m_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("wfs_kernels.hip", "regfft.h", "noise.h", "internal.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(frames_per_launch):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary, or None if the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_frame = (t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]) / t["frames_per_launch"]
    return per_frame * frames_per_launch


def cpu_baseline(cfg, launch, opd, min_seconds=10.0):
    """The FP64 oracle on a bounded sample: every 4th valid sub-aperture of each sensor, repeated
    until min_seconds of CPU time have been spent; scaled to whole frames/s."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import wfs as OW

    sens = OW.Sensor(cfg, 6, launch)
    sub = np.arange(0, sens.n_valid, 4)
    for w in range(6):
        sens.khat(w, sub)               # plan setup, outside the timed region
    reps = 0
    t0 = time.perf_counter()
    while True:
        sens.measure(opd[:1], seed=698, frame0=0, subset=sub)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    per_frame = el / reps * (sens.n_valid / len(sub))
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": 1.0 / per_frame, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(sub)} of {sens.n_valid} sub-apertures of each of the 6 sensors (every 4th), "
                      f"noise on, {reps} repetitions in {el:.1f} s, scaled to whole frames; kernel spectra "
                      f"computed before timing"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames-per-step", type=int, default=1)
    ap.add_argument("--resident-frames", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, run 5 plain device copies of this many MB (profiler counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs

    torch.cuda.set_device(0)
    cfg = G.CFG1
    launch = G.launch_positions(cfg, 6)
    plan = shwfs.WfsPlan(cfg, 6, launch)
    B = args.frames_per_step
    nres = max(args.resident_frames, B)
    opd_host = S.lgs39m_opd(nres, 6)
    opd = torch.from_numpy(opd_host).cuda()
    slopes = torch.zeros((B, 6, 2, plan.n_valid), device="cuda")
    stream = torch.cuda.current_stream()

    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(k):
        f0 = (k * B) % (nres - B + 1)
        plan.measure(opd[f0:f0 + B], slopes, seed=G.NOISE_SEED, frame0=k * B, stream=stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step(args.warmup + k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])      # ms per launch (B frames)
    frames = args.steps * B
    value = frames / wall
    avg_launch_ms = float(lat.mean())
    subaps = 6 * plan.n_valid * B
    achieved = FLOP_PER_SUBAP * subaps / (avg_launch_ms * 1e-3) / 1e12
    out = {
        "metric": "SH-WFS frames/s (6 LGS, 80x80 subaps)",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lgs39m: 6 LGS SH-WFS, 800x800 pupil at 4.875e-2 m, 80x80 subaps of 10x10 px, "
                               "FFT 40, sodium kernel, 16x16 det px, 500 ph + 3 e- RON, threshold 3 e-",
                   "frames_per_step": B, "subaps_per_frame": 6 * plan.n_valid},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "per": f"launch of {B} frame(s), HIP events on the launch stream"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(B),
                     "kernel": "wfs_fused_kernel<10,40,40,16,lgs>",
                     "avg_launch_ms": avg_launch_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, launch, opd_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
