#!/usr/bin/env python3
"""Benchmark of the local bundle adjustment hot path on one MI355X.

One step = one complete solve (round 1: 5 LM iterations, chi-square outlier pass,
round 2: 10 LM iterations, final flags) of the workload's window(s), inputs already
resident in device memory.  The reported value is window-LM-iterations per second over
the timed steps.  Per-kernel durations come from HIP events the library records around
every launch on the solve's stream during the timed steps; the dominant kernel's
algorithmic bytes (or flops) per launch divided by its mean launch time give the roofline
entry.  The CPU baseline is the FP64 oracle timed on this host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Local BA LM iter/s + residual/Hessian HBM GB/s; FP32/batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "c2_stereo_fp64": dict(
        desc="plain FP64 stereo local BA, seed 1: 20 optimisable + 10 fixed keyframes on a 6 m "
             "random walk, 8,000 points 1-12 m deep, 8 observations per point (70% stereo), "
             "5% outliers, 5+10 LM iterations",
        precision="fp64"),
}


def make_data(name):
    from paper_2511_02036_amd import synth
    if name == "c2_stereo_fp64":
        return [synth.c2_stereo(seed=1)]
    raise ValueError(name)


def kernel_bytes_and_flops(cls, w, n_tiles, real_bytes, z_bytes):
    """Algorithmic bytes and flops of ONE launch of a kernel class for one window shape
    (w: dict with K, M, N, Kopt, stereo share).  Bytes count what the kernel must read
    and write once: observation records, point states, poses, and its outputs."""
    K, M, N, n = w["K"], w["M"], w["N"], 6 * w["Kopt"]
    E = n * (n + 1) // 2
    obs_rec = 4 + 4 + 3 * z_bytes + 1 + 1          # kf, pt, u/v/uR, type, octave
    if cls == "linearize":
        b = N * obs_rec + M * (24 + 4) + n_tiles * (K * 100 + (E + 2 * n) * real_bytes + 32)
        # residual+Jacobian+blocks ~420 flop/obs, point factor ~60 flop/point,
        # Schur pairs 216 flop per ordered pair of a point's optimisable observations
        f = 420 * N + 60 * M + 216 * w["pairs"]
        return b, f
    if cls == "update":
        b = N * obs_rec + M * (24 + 24 + 4) + n_tiles * (K * 100 + n * 8 + 32)
        f = 330 * N + 60 * M
        return b, f
    if cls == "reduce":
        return n_tiles * (E + 2 * n) * real_bytes + (E + 2 * n) * 8, n_tiles * (E + 2 * n)
    if cls == "cholesky":
        return (E + 2 * n) * 8 + n * 8, n ** 3 / 3 + 2 * n * n
    return 0, 0


def window_shape(w):
    import numpy as np
    N = len(w["obs_kf"])
    opt = w["fixed"] == 0
    on_opt = opt[w["obs_kf"]]
    cnt = np.bincount(w["obs_pt"][on_opt], minlength=len(w["X"]))
    pairs = int((cnt * cnt).sum())
    return dict(K=len(w["fixed"]), M=len(w["X"]), N=N, Kopt=int(opt.sum()), pairs=pairs)


def cpu_baseline(windows, budget_s=12.0):
    """Time the FP64 CPU oracle (single thread) on a bounded sample of the workload."""
    from oracle import lbaref
    t0 = time.perf_counter()
    iters = 0
    runs = 0
    while True:
        for w in windows:
            r = lbaref.solve(w)
            iters += int(r["stats"]["iters_r1"] + r["stats"]["iters_r2"])
            runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return dict(value=iters / el, unit="window-LM-iterations/s", cores=1, kind="oracle",
                sample=f"{runs} full solves of the benchmark window(s) in {el:.1f} s, one thread",
                seconds=el), r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2_stereo_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the windows are independent, see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2511_02036_amd import lba, synth

    spec = WORKLOADS[args.workload]
    windows = make_data(args.workload)
    data = windows[0] if len(windows) == 1 else synth.concat(windows)
    mixed = spec["precision"] == "mixed"
    z_f32 = spec.get("z_f32", False)
    dev = torch.device("cuda:0")
    ctx = lba.Context(device=0, precision=spec["precision"])
    prob = lba.DeviceProblem(data, device=dev, z_f32=z_f32)
    solver = lba.Solver(ctx, prob)
    stream = torch.cuda.current_stream(dev)

    print(f"bench: workload={args.workload} windows={len(windows)} obs={prob.obs_kf.shape[0]} "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        solver.run(stream)
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(args.steps):
        solver.run(stream)
        iters += int(solver.stats[:, 2].sum() + solver.stats[:, 3].sum())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    print(f"bench: timed {args.steps} steps in {el:.3f} s", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel --------------------------------------------
    shapes = [window_shape(w) for w in windows]
    real_bytes = 4 if mixed else 8
    z_bytes = 4 if z_f32 else 8
    kern = {k: dict(launches=n, total_ms=ms, mean_us=(1e3 * ms / n if n else 0.0)) for k, (n, ms) in prof.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    # tiles per window follow the library's plan (same rule as the C++ planner)
    ppt = tile_points(sum(s["M"] for s in shapes))
    tot_b = tot_f = 0.0
    for s in shapes:
        b, f = kernel_bytes_and_flops(dom, s, (s["M"] + ppt - 1) // ppt, real_bytes, z_bytes)
        tot_b += b
        tot_f += f
    mean_s = kern[dom]["mean_us"] * 1e-6
    if dom == "cholesky":
        peak = FP64_PEAK_TFLOPS
        ach = tot_f / mean_s / 1e12 if mean_s > 0 else 0.0
        roof = dict(kernel=dom, bound="alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=None, flops_per_launch=tot_f)
    else:
        ach = tot_b / mean_s / 1e9 if mean_s > 0 else 0.0
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None, bytes_per_launch=tot_b, mean_us=kern[dom]["mean_us"])

    out = {
        "metric": METRIC,
        "value": iters / el,
        "unit": "window-LM-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": spec["desc"], "windows": len(windows),
                   "keyframes": int(sum(s["K"] for s in shapes)), "points": int(sum(s["M"] for s in shapes)),
                   "observations": int(sum(s["N"] for s in shapes)), "lm_iterations_per_step": iters // args.steps},
        "roofline": roof,
        "kernels_us_mean": {k: round(v["mean_us"], 2) for k, v in kern.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        cb, last = cpu_baseline(windows)
        out["cpu_baseline"] = cb
        # the last oracle solve doubles as a parity spot check of the benchmark window
        g = solver.stats[0]
        out["parity_final_cost_rel"] = abs(g[1] - last["stats"]["F_final"]) / abs(last["stats"]["F_final"])
    print(json.dumps(out), flush=True)


def tile_points(total_points):
    """Points per tile as the library's planner picks them by default."""
    p = (total_points + 1023) // 1024
    p = (p + 31) // 32 * 32
    return max(64, min(4096, p))


if __name__ == "__main__":
    main()
