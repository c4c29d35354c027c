#!/usr/bin/env python3
"""Benchmark of the local bundle adjustment hot path on one MI355X.

One step = one complete solve (round 1: 5 LM iterations, chi-square outlier pass,
round 2: 10 LM iterations, final flags) of the workload's window(s), inputs already
resident in device memory.  The reported value is window-LM-iterations per second over
the timed steps.

Default workload: the 256-window batch (uneven windows shaped like stereo local maps)
solved in one batched call in mixed precision (FP32 Jacobians / Hessian blocks / Schur,
FP64 Cholesky, cost, gain ratio, damping and states).  Beside it the same 256 windows
are solved one call per window in plain FP64 (the comparison the metric names).

Per-kernel durations come from HIP events the library records around every launch on
the solve's stream during the timed steps; the dominant kernel's algorithmic bytes and
flops per launch divided by its mean launch time give the roofline entry.  The CPU
baseline is the FP64 oracle timed on this host on a bounded sample of the workload.

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
# published MI355X vector peaks: FP32 157.3 TFLOP/s (256 CUs x 2.4 GHz x 256 flop/clock,
# which needs packed FP32 FMAs) and FP64 78.6 TFLOP/s.  The library is built without packed
# FP32 instructions, so its FP32 code issues at the FP64 / non-packed rate of 78.6; that
# figure is reported beside the published one.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
NONPACKED_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "c5_batched_mixed": dict(
        desc="256 local windows of uneven size (seed 4): keyframes U{5..40} with a third fixed, "
             "points U{500..20000}, 4-10 observations per point, 70/30 stereo/mono, 5% outliers; "
             "one batched solve per step, FP32 bulk + FP64 reduced solve, FP32 measurements, "
             "5+10 LM iterations",
        precision="mixed", z_f32=True, compare_plain=True),
    "c5_batched_fp64": dict(
        desc="the 256-window batch (seed 4) solved in one batched call in plain FP64",
        precision="fp64", z_f32=False, compare_plain=False),
    "c2_stereo_fp64": dict(
        desc="plain FP64 stereo local BA, seed 1: 20 optimisable + 10 fixed keyframes on a 6 m "
             "random walk, 8,000 points 1-12 m deep, 8 observations per point (70% stereo), "
             "5% outliers, 5+10 LM iterations",
        precision="fp64", z_f32=False, compare_plain=False),
    "c1_mono_fp64": dict(
        desc="plain FP64 monocular local BA, seed 0: 10 optimisable + 5 fixed keyframes on a 2 m arc, "
             "1,500 points, 8 observations per point, 5+10 LM iterations",
        precision="fp64", z_f32=False, compare_plain=False),
    "c4_differentiation": dict(
        desc="differentiation form, seed 3: 64 windows of 10 keyframes and 2,000 points, 8 observations "
             "per point, even windows monocular, odd 70/30 stereo/mono; one step = FP32 robust-cost "
             "forward + hand-written backward (gradients for poses, points, measurements) of all windows",
        precision="fp64", z_f32=True, compare_plain=False),
    "corr_search": dict(
        desc="keypoint correspondence search (map-point creation), seed 5: GPU-resident keyframe store of "
             "80 keyframes x 1,200 keypoints (256-bit descriptors, octaves U{0..7}, 70% stereo, 60% without "
             "a map point), the last 64 keyframes each against its 10 nearest: 640 keyframe pairs per step",
        precision="i8+f64", z_f32=False, compare_plain=False),
    "fusion_search": dict(
        desc="map-point fusion candidate search, seeds 5 and 6: the same store; the map points of the last 64 "
             "keyframes (about 390 each) against each keyframe's 20 nearest: 1,280 queries, about 496k "
             "point-keyframe pairs per step",
        precision="f64", z_f32=False, compare_plain=False),
    "culling_batched": dict(
        desc="keyframe-culling counters over the observations of the 256-window batch (seed 4; 18M "
             "observations, 2.6M points, 5,700 keyframes, global indices, every 13th observation inactive)",
        precision="i32", z_f32=False, compare_plain=False),
    "vi_stereo_fp64": dict(
        desc="stereo-inertial local BA, seed 7: 10 optimisable + 5 fixed keyframes on a 4 m walk with "
             "preintegrated IMU measurements between consecutive keyframes, 6,000 points, 8 observations per "
             "point (70% stereo), 5% outliers; FP64, 15 unknowns per keyframe (joint reduced system of 150), "
             "5+10 LM iterations",
        precision="fp64", z_f32=False, compare_plain=False),
    "vi_batched_mixed": dict(
        desc="64 stereo-inertial windows (seed 8): keyframes U{6..15} with a third fixed (at most 12 "
             "optimisable), points U{1,000..8,000}, 4-10 observations per point, 70/30 stereo/mono, IMU "
             "measurements between consecutive keyframes; one batched solve per step, FP32 visual bulk + FP64 "
             "inertial terms and reduced solve, 5+10 LM iterations",
        precision="mixed", z_f32=True, compare_plain=False),
    "c3_precision_mixed": dict(
        desc="precision form, seed 2: 30 optimisable + 20 fixed stereo keyframes, 20,000 points, "
             "10 observations per point, FP32 bulk + FP64 reduced solve, 5+10 LM iterations",
        precision="mixed", z_f32=True, compare_plain=False),
}


def make_windows(name):
    from paper_2511_02036_amd import synth
    if name.startswith("c5"):
        return synth.c5_windows(seed=4)
    if name.startswith("c2"):
        return [synth.c2_stereo(seed=1)]
    if name.startswith("c1"):
        return [synth.c1_mono(seed=0)]
    if name.startswith("c3"):
        return [synth.c3_precision(seed=2)]
    if name.startswith("c4"):
        return synth.c4_windows(seed=3)
    raise ValueError(name)


def window_shape(w):
    import numpy as np
    opt = w["fixed"] == 0
    on_opt = opt[w["obs_kf"]]
    cnt = np.bincount(w["obs_pt"][on_opt], minlength=len(w["X"]))
    st = np.asarray(w["obs_type"]).astype(bool)
    return dict(K=len(w["fixed"]), M=len(w["X"]), N=len(w["obs_kf"]), Kopt=int(opt.sum()),
                N_stereo=int(st.sum()), pairs=int((cnt * (cnt - 1) // 2).sum()), self_terms=int(cnt.sum()))


# Algorithmic work per unit, from the scope table's measurement section (per observation
# per LM step, FP32 bulk): the observation record is 22 B (u, v, uR 12 + keyframe 4 +
# point 4 + octave 1 + type 1; 34 B with FP64 measurements); residual + Jacobian + block
# Hessian 300 flops (mono) / 420 (stereo); the Schur complement 440 flops; the trial cost
# 40.  A point's FP64 position is 24 B, read once per linearisation and read + written
# once per update.
FLOP_RES_HESS = {False: 300, True: 420}
FLOP_SCHUR = 440
FLOP_TRIAL = 40


def kernel_bytes_and_flops(cls, s, z_bytes):
    """Algorithmic bytes and flops of ONE launch of a kernel class over one window of
    shape s: the per-unit figures above times the observations and points one launch
    processes (every observation of the window: the masked round-2 outliers are read too)."""
    M, N, Ns = s["M"], s["N"], s["N_stereo"]
    obs_rec = 4 + 4 + 3 * z_bytes + 1 + 1
    res_hess = FLOP_RES_HESS[False] * (N - Ns) + FLOP_RES_HESS[True] * Ns
    if cls == "linearize":
        return N * obs_rec + M * 24, res_hess + FLOP_SCHUR * N
    if cls == "update":
        return N * obs_rec + M * 48, FLOP_TRIAL * N
    if cls == "linearize_init":
        return N * obs_rec + M * 24, res_hess
    if cls == "cholesky":
        # the reduced system of n = 6 Kopt unknowns: factorisation n^3 / 3 plus the forward and
        # back solves 2 n^2 flops (FP64), its packed triangle and right side read once
        n = 6 * s["Kopt"]
        return 8 * (n * (n + 1) // 2 + n), n ** 3 / 3.0 + 2.0 * n * n
    return 0, 0


def copy_peak_gbs(dev, mib=1024, reps=10):
    """Device-to-device copy rate of this GPU (bytes read + written per second, best of
    three timed groups of `reps` copies of `mib` MiB): the HBM rate a plain stream reaches
    here, reported beside the published 8 TB/s."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            dst.copy_(src)
        b.record()
        b.synchronize()
        t = a.elapsed_time(b) * 1e-3
        best = t if best is None else min(best, t)
    del src, dst
    return 2.0 * (mib << 20) * reps / best / 1e9


def kernel_roofs(cls, shapes, mean_us, mixed, z_f32):
    tb = tf = 0.0
    for s in shapes:
        b, f = kernel_bytes_and_flops(cls, s, 4 if z_f32 else 8)
        tb += b
        tf += f
    sec = mean_us * 1e-6
    gbs = tb / sec / 1e9 if sec > 0 else 0.0
    tfs = tf / sec / 1e12 if sec > 0 else 0.0
    peak = FP32_PEAK_TFLOPS if (mixed and cls != "cholesky") else FP64_PEAK_TFLOPS
    return dict(bytes_per_launch=tb, flops_per_launch=tf, mean_us=mean_us, achieved_GBs=gbs,
                hbm_frac=gbs / HBM_PEAK_GBS, achieved_TFLOPs=tfs, alu_peak=peak, alu_frac=tfs / peak,
                alu_frac_nonpacked=tfs / NONPACKED_PEAK_TFLOPS)


def code_text(path):
    """A source file with its comments and blank lines removed, each line stripped: the
    key of a counter record, so that comment edits do not retire measured traffic."""
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(l.strip() for l in src.splitlines() if l.strip())


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of this workload
    (profiles/<workload>_traffic.md), or None when there is none or the kernel's source has
    changed since the counters were taken."""
    import hashlib
    src = {"linearize": "k_linearize.hip", "update": "k_update.hip", "cost_forward": "k_cost.hip",
           "cost_backward": "k_cost.hip"}.get(kernel)
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.md")
    if src is None or not os.path.exists(path):
        return None
    h = hashlib.sha256(code_text(os.path.join(ROOT, "paper_2511_02036_amd", "csrc", src)).encode()).hexdigest()[:16]
    with open(path) as f:
        for line in f:
            w = line.split()
            if len(w) == 5 and w[0] == "traffic" and w[1] == "k_" + kernel and w[3] == "code-sha256":
                return float(w[2]) if w[4] == h else None
    return None


def host_description():
    """CPU model, logical CPUs of the host (nproc) and CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return dict(cpu_model=model, nproc=os.cpu_count() or 1, cpus_allowed=allowed)


# threads of the oracle pool: the host's CPUs, at most 16 (the CPU share of one GPU on
# the hosts this runs on)
MAX_POOL = 16


def cpu_baseline(windows, budget_s=12.0, single_budget_s=8.0, z_f32=False):
    """The FP64 CPU oracle on a bounded sample of the workload's windows: a thread pool
    over the host cores for batches (plus a one-thread figure on the first windows), one
    thread for a single window.  Returns the baseline record and {window index: oracle
    result} of the windows the pool solved."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import lbaref
    host = host_description()
    if z_f32:
        # the oracle reads the measurements the GPU read (FP32-rounded), so that its results
        # double as the parity reference of the benchmarked solve
        from tests.parity import round_z_f32
        windows = [round_z_f32(w) for w in windows]
    if len(windows) == 1:
        t0 = time.perf_counter()
        iters = runs = 0
        last = None
        while True:
            last = lbaref.solve(windows[0])
            iters += int(last["stats"]["iters_r1"] + last["stats"]["iters_r2"])
            runs += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
        return dict(value=iters / el, unit="window-LM-iterations/s", cores=1, kind="oracle",
                    sample=f"{runs} full solves of the benchmark window in {el:.1f} s, one thread",
                    **host), {0: last}
    cores = max(1, min(MAX_POOL, host["cpus_allowed"]))
    # estimate per-window cost from observation counts; take windows in batch order until
    # about budget_s of CPU time on the pool
    per_obs_s = 4.5e-6
    n = 0
    acc = 0.0
    while n < len(windows) and acc < budget_s * cores:
        acc += per_obs_s * len(windows[n]["obs_kf"])
        n += 1
    sample = list(range(n))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(lambda i: lbaref.solve(windows[i]), sample))
    el = time.perf_counter() - t0
    iters = sum(int(r["stats"]["iters_r1"] + r["stats"]["iters_r2"]) for r in res)
    nobs = sum(len(windows[i]["obs_kf"]) for i in sample)
    # one thread on the first windows of the batch, about single_budget_s
    t1 = time.perf_counter()
    it1 = n1 = ob1 = 0
    while n1 < len(windows) and time.perf_counter() - t1 < single_budget_s:
        r = lbaref.solve(windows[n1])
        it1 += int(r["stats"]["iters_r1"] + r["stats"]["iters_r2"])
        ob1 += len(windows[n1]["obs_kf"])
        n1 += 1
    el1 = time.perf_counter() - t1
    return dict(value=iters / el, unit="window-LM-iterations/s", cores=cores, kind="oracle",
                sample=f"first {n} of {len(windows)} windows ({nobs} observations), one window per "
                       f"thread on {cores} threads, {el:.1f} s",
                one_core=dict(value=it1 / el1, sample=f"first {n1} windows ({ob1} observations) in "
                                                      f"{el1:.1f} s on one thread"),
                **host), dict(zip(sample, res))


def cost_layer_bytes(cls, windows):
    """Algorithmic bytes and flops of one launch of the robust-cost layer over all windows:
    forward reads each observation record (22 B) and each point (12 B); backward also
    writes 12 B of measurement gradient per observation and 12 B of point gradient per
    point.  Flops: ~45 per observation forward, ~110 backward (counted from the kernel)."""
    N = sum(len(w["obs_kf"]) for w in windows)
    M = sum(len(w["X"]) for w in windows)
    if cls == "cost_forward":
        return N * 22 + M * 16, 45 * N
    return N * 34 + M * 28, 110 * N


def bench_cost_layer(args, spec):
    """One step = forward + backward of the robust-cost layer over every window."""
    import numpy as np
    import torch
    from paper_2511_02036_amd import lba, synth
    windows = make_windows(args.workload)
    cat = synth.concat(windows)
    dev = torch.device("cuda:0")
    ctx = lba.Context(device=0, check_inputs=0)
    layer = lba.CostLayer(ctx, cat, device=dev)
    X = torch.tensor(np.asarray(cat["X"], dtype=np.float32).reshape(-1, 3), device=dev)
    z = torch.tensor(np.asarray(cat["obs_z"], dtype=np.float32).reshape(3, -1), device=dev)
    xi = torch.zeros((layer.n_kf, 6), dtype=torch.float32, device=dev)
    g = torch.ones(layer.n_windows, dtype=torch.float64, device=dev)
    def step():
        layer.forward(xi, X, z)
        layer.backward(xi, X, z, g)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps, 1) * 20
    # per-kernel HIP events (each call then waits for its kernels): kernel means only
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    pel = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    # the timed steps: calls enqueue their work and return, as in use
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = {k: dict(launches=n, mean_us=(1e3 * ms / n if n else 0.0)) for k, (n, ms) in prof.items() if n}
    b, f = cost_layer_bytes("cost_backward", windows)
    mb = kern["cost_backward"]["mean_us"] * 1e-6
    roof = dict(kernel="cost_backward", bound="hbm", achieved=b / mb / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=b / mb / 1e9 / HBM_PEAK_GBS, traffic=measured_traffic(args.workload, "cost_backward"), bytes_per_launch=b, mean_us=kern["cost_backward"]["mean_us"],
                alu_TFLOPs=f / mb / 1e12)
    cp = copy_peak_gbs(dev)
    roof["copy_peak_GBs"] = cp
    roof["frac_of_copy_peak"] = b / mb / 1e9 / cp
    nw = len(windows)
    out = {"metric": METRIC, "value": nw * steps / el, "unit": "window-cost-gradients/s", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "description": spec["desc"], "windows": nw,
                      "observations": int(sum(len(w["obs_kf"]) for w in windows)),
                      "points": int(sum(len(w["X"]) for w in windows))},
           "roofline": roof, "kernels_us_mean": {k: round(v["mean_us"], 2) for k, v in kern.items()},
           "profiled": {"ms_per_step": 1e3 * pel / steps,
                        "note": "the same steps with per-kernel HIP events, where every call waits for its "
                                "kernels (kernel means above come from this pass)"}}
    if not args.no_cpu_baseline:
        from oracle import lbaref
        t0 = time.perf_counter()
        n = 0
        while True:
            lbaref.cost_grad(windows[n % nw])
            n += 1
            if time.perf_counter() - t0 >= 10.0:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=n / el, unit="window-cost-gradients/s", cores=1, kind="oracle",
                                   sample=f"{n} FP64 cost + gradient evaluations of the workload's windows "
                                          f"in {el:.1f} s, one thread")
    print(json.dumps(out), flush=True)


# dense int8 matrix-core peak of MI355X (published; no sparsity)
INT8_PEAK_TOPS = 5000.0


def map_search_job(name):
    """(job, per-launch work record, oracle sample runner) of a local-mapping workload."""
    import numpy as np
    from paper_2511_02036_amd import lmap, synth
    if name == "culling_batched":
        wins = synth.c5_windows(seed=4)
        kf, pt, oc = [], [], []
        k0 = p0 = 0
        for w in wins:
            kf.append(w["obs_kf"] + k0)
            pt.append(w["obs_pt"] + p0)
            oc.append(w["obs_oct"])
            k0 += len(w["fixed"])
            p0 += len(w["X"])
        kf, pt, oc = np.concatenate(kf), np.concatenate(pt), np.concatenate(oc)
        active = np.ones(len(kf), np.uint8)
        active[::13] = 0
        job = lmap.Culling(k0, p0, kf, pt, oc, active=active)
        n_obs, n_pt = len(kf), p0
        work = dict(kind="culling", n_obs=n_obs, n_pt=n_pt, n_kf=k0,
                    # count: point, octave, flag (6 B) per observation + one 4-byte counter add;
                    # redundancy: keyframe, point, octave, flag (10 B) + the point's 8 counters
                    bytes={"cull_count": n_obs * 10 + n_pt * 8 * 4,
                           "cull_redundant": n_obs * 10 + n_pt * 8 * 4 + k0 * 8})

        def oracle_sample(budget_s):
            from oracle import mapref
            order = np.argsort([len(w["obs_kf"]) for w in wins])
            t0 = time.perf_counter()
            n = obs = 0
            while n < len(order) and time.perf_counter() - t0 < budget_s:
                w = wins[order[n]]
                mapref.culling(w)
                obs += len(w["obs_kf"])
                n += 1
            el = time.perf_counter() - t0
            return obs / el, f"the {n} smallest of the 256 windows ({obs} observations) in {el:.1f} s, one thread"
        return job, work, oracle_sample, "observations/s", n_obs
    st = synth.keyframe_store()
    ds = lmap.DeviceStore(st)
    if name == "corr_search":
        cur, nbr = synth.correspondence_queries(st)
        job = lmap.Correspondence(ds, cur, nbr)
        free = ds.upload_free(st["kp_free"])
        ko, fr = st["kp_off"], st["kp_free"].astype(np.int64)
        nfree = np.array([fr[ko[k]:ko[k + 1]].sum() for k in range(len(ko) - 1)])
        pairs = int((nfree[cur] * nfree[nbr]).sum())
        work = dict(kind="corr", pairs=pairs, ops=2 * 256 * pairs, queries=len(cur))
        run = lambda: job.run(free, check=False)

        def oracle_sample(budget_s):
            from oracle import mapref
            t0 = time.perf_counter()
            n = 0
            while n < len(cur) and time.perf_counter() - t0 < budget_s:
                mapref.correspondence(st, cur[n:n + 4], nbr[n:n + 4])
                n += 4
            el = time.perf_counter() - t0
            return n / el, f"the first {n} of {len(cur)} keyframe pairs in {el:.1f} s, one thread"
        job.run_step = run
        return job, work, oracle_sample, "keyframe-pairs/s", len(cur)
    pts, q = synth.fusion_points(st)
    job = lmap.Fusion(ds, pts, q)
    entries = int(np.sum(q[1] - q[0]))
    # per (point, keyframe) entry: the point's position, direction, range and descriptor
    # (24 + 24 + 16 + 32 B) and its two outputs (8 B); per query the keyframe's pose (96 B)
    work = dict(kind="fusion", entries=entries, bytes={"fuse": entries * 104 + len(q[0]) * 96})

    def oracle_sample(budget_s):
        from oracle import mapref
        t0 = time.perf_counter()
        n = 0
        while n < len(q[0]) and time.perf_counter() - t0 < budget_s:
            sl = slice(n, n + 20)
            mapref.fusion(st, pts, (q[0][sl], q[1][sl], q[2][sl]))
            n += 20
        el = time.perf_counter() - t0
        done = int(np.sum(q[1][:n] - q[0][:n]))
        return done / el, f"the first {n} of {len(q[0])} queries ({done} point-keyframe pairs) in {el:.1f} s, one thread"
    return job, work, oracle_sample, "point-keyframe-pairs/s", entries


def bench_map_search(args, spec):
    """One step = one call of the search over the whole workload, inputs resident on the GPU."""
    import torch
    from paper_2511_02036_amd import lmap
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    job, work, oracle_sample, unit, units_per_step = map_search_job(args.workload)
    step = getattr(job, "run_step", None) or (lambda: job.run(check=False))
    print(f"bench: workload={args.workload} set up in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps, 1) * 10
    lmap.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    pel = time.perf_counter() - t0
    prof = lmap.profile_read()
    lmap.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = {k: dict(launches=n, mean_us=1e3 * ms / n) for k, (n, ms) in prof.items() if n}
    if work["kind"] == "corr":
        mu = kern["corr_search"]["mean_us"]
        tops = work["ops"] / (mu * 1e-6) / 1e12
        roof = dict(kernel="corr_search", bound="mfma", achieved=tops, peak=INT8_PEAK_TOPS, unit="TOP/s",
                    frac=tops / INT8_PEAK_TOPS, traffic=None, ops_per_launch=work["ops"],
                    keypoint_pairs_per_launch=work["pairs"], mean_us=mu,
                    note="int8 products of the +-1 descriptor bytes: 2 x 256 operations per pair of free "
                         "keypoints (the pairs the search must compare)")
    else:
        dom = max(work["bytes"], key=lambda k: kern.get(k, {"mean_us": 0})["mean_us"])
        mu = kern[dom]["mean_us"]
        gbs = work["bytes"][dom] / (mu * 1e-6) / 1e9
        roof = dict(kernel=dom, bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                    traffic=None, bytes_per_launch=work["bytes"][dom], mean_us=mu)
    out = {"metric": f"{args.workload}: {unit}", "value": units_per_step * steps / el, "unit": unit, "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": spec["precision"], "data": "synthetic",
           "config": {"workload": args.workload, "description": spec["desc"],
                      **{k: v for k, v in work.items() if k not in ("bytes", "kind")}},
           "roofline": roof, "kernels_us_mean": {k: round(v["mean_us"], 2) for k, v in kern.items()},
           "profiled": {"ms_per_step": 1e3 * pel / steps,
                        "note": "the same steps with per-kernel HIP events (each call then waits for its kernels)"}}
    if not args.no_cpu_baseline:
        v, sample = oracle_sample(10.0)
        out["cpu_baseline"] = dict(value=v, unit=unit, cores=1, kind="oracle", sample=sample, **host_description())
    print(json.dumps(out), flush=True)


def inertial_windows(name):
    from paper_2511_02036_amd import synth
    import numpy as np
    if name == "vi_stereo_fp64":
        return [synth.vi_stereo(seed=7)]
    out = []
    for i, ss in enumerate(np.random.SeedSequence(8).spawn(64)):
        rng = np.random.default_rng(ss)
        K = int(rng.integers(6, 16))
        M = int(rng.integers(1000, 8001))
        out.append(synth.vi_window(int(rng.integers(0, 2 ** 31)), K=K, n_fixed=max(K // 3, K - 12), M=M,
                                   nobs=(4, 10), stereo_p=0.7, walk_length=0.3 * K))
    return out


def bench_inertial(args, spec):
    """One step = one stereo-inertial solve (lba_solve_inertial) of the workload."""
    import numpy as np
    import torch
    from paper_2511_02036_amd import lba, synth
    pairs = inertial_windows(args.workload)
    w, vi = pairs[0] if len(pairs) == 1 else synth.concat_vi(pairs)
    dev = torch.device("cuda:0")
    ctx = lba.Context(device=0, precision=spec["precision"])
    prob = lba.DeviceProblem(w, device=dev, z_f32=spec["z_f32"])
    dvi = lba.DeviceInertial(vi, device=dev)
    solver = lba.InertialSolver(ctx, prob, dvi)
    stream = torch.cuda.current_stream(dev)
    for _ in range(max(args.warmup, 1)):
        solver.run(stream)
    torch.cuda.synchronize()
    steps = max(args.steps, 1)
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.run(stream)
    torch.cuda.synchronize()
    pel = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    solver.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(steps):
        solver.run(stream)
        iters += int(solver.stats[:, 2].sum() + solver.stats[:, 3].sum())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = {k: dict(launches=n, mean_us=1e3 * ms / n) for k, (n, ms) in prof.items() if n}
    shapes = [window_shape(p[0]) for p in pairs]
    mixed = spec["precision"] == "mixed"
    r = kernel_roofs("linearize", shapes, kern["linearize"]["mean_us"], mixed, spec["z_f32"])
    if r["alu_frac"] >= r["hbm_frac"]:
        roof = dict(kernel="linearize", bound="alu", achieved=r["achieved_TFLOPs"], peak=r["alu_peak"],
                    unit="TFLOP/s", frac=r["alu_frac"], traffic=None, mean_us=r["mean_us"],
                    flops_per_launch=r["flops_per_launch"], hbm_frac=r["hbm_frac"])
    else:
        roof = dict(kernel="linearize", bound="hbm", achieved=r["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=r["hbm_frac"], traffic=None, mean_us=r["mean_us"], bytes_per_launch=r["bytes_per_launch"])
    out = {"metric": METRIC, "value": iters / el, "unit": "window-LM-iterations/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
           "config": {"workload": args.workload, "description": spec["desc"], "windows": len(pairs),
                      "keyframes": int(sum(s["K"] for s in shapes)), "points": int(sum(s["M"] for s in shapes)),
                      "observations": int(sum(s["N"] for s in shapes)),
                      "inertial_measurements": int(len(vi["dt"])),
                      "lm_iterations_per_step": iters // steps},
           "roofline": roof, "kernels_us_mean": {k: round(v["mean_us"], 2) for k, v in kern.items()},
           "profiled": {"ms_per_step": 1e3 * pel / steps,
                        "note": "the same steps with per-kernel HIP events, kernels launched one by one"}}
    if not args.no_cpu_baseline:
        from oracle import lbaref
        zr = (lambda x: x)
        if spec["z_f32"]:
            from tests.parity import round_z_f32
            zr = round_z_f32
        t0 = time.perf_counter()
        it = n = 0
        res = {}
        while n < len(pairs) and time.perf_counter() - t0 < 10.0:
            rr = lbaref.solve_vi(zr(pairs[n][0]), pairs[n][1])
            res[n] = rr
            it += int(rr["stats"]["iters_r1"] + rr["stats"]["iters_r2"])
            n += 1
        cel = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=it / cel, unit="window-LM-iterations/s", cores=1, kind="oracle",
                                   sample=f"the first {n} of {len(pairs)} windows in {cel:.1f} s, one thread",
                                   **host_description())
        rel = [abs(solver.stats[i, 1] - rr["stats"]["F_final"]) / abs(rr["stats"]["F_final"]) for i, rr in res.items()]
        out["parity"] = {"windows_checked": len(rel), "final_cost_rel_max": float(max(rel))}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5_batched_mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-window plain FP64 comparison")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile tuner")
    ap.add_argument("--fp32-accum", action="store_true",
                    help="mixed workloads: sum the Schur complement in FP32 (the literal precision form)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device to device once (a kernel of known traffic that "
                         "calibrates hardware byte counters read by a profiler)")
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
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload.startswith("c4"):
        bench_cost_layer(args, spec)
        return
    if args.workload in ("corr_search", "fusion_search", "culling_batched"):
        bench_map_search(args, spec)
        return
    if args.workload.startswith("vi_"):
        bench_inertial(args, spec)
        return
    t_gen = time.perf_counter()
    windows = make_windows(args.workload)
    data = windows[0] if len(windows) == 1 else synth.concat(windows)
    mixed = spec["precision"] == "mixed"
    z_f32 = spec["z_f32"]
    dev = torch.device("cuda:0")
    ctx = lba.Context(device=0, precision=spec["precision"], schur_fp32_accum=1 if args.fp32_accum else 0)
    prob = lba.DeviceProblem(data, device=dev, z_f32=z_f32)
    stream = torch.cuda.current_stream(dev)
    tuned = None
    if not args.no_tune:
        # the tile tuner (short solves; its table is kept in the context)
        t_tune = time.perf_counter()
        tuned = ctx.tune(prob, stream)
        print(f"bench: tile table {tuned} tuned in {time.perf_counter() - t_tune:.1f} s", file=sys.stderr, flush=True)
    solver = lba.Solver(ctx, prob)
    print(f"bench: workload={args.workload} windows={len(windows)} obs={prob.obs_kf.shape[0]} "
          f"(generated in {time.perf_counter() - t_gen:.1f} s) warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        solver.run(stream)
    torch.cuda.synchronize()
    # two small tagged kernels bracket the timed steps in a profiler's kernel trace
    marker = torch.ones(1, device=dev)
    marker.mul_(3.0)
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
    marker.div_(3.0)
    torch.cuda.synchronize()
    print(f"bench: timed {args.steps} steps in {el:.3f} s", file=sys.stderr, flush=True)
    # the same steps again without per-kernel events: each LM step replays its captured graph
    solver.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    giters = 0
    for _ in range(args.steps):
        solver.run(stream)
        giters += int(solver.stats[:, 2].sum() + solver.stats[:, 3].sum())
    torch.cuda.synchronize()
    gel = time.perf_counter() - t0

    shapes = [window_shape(w) for w in windows]
    kern = {k: dict(launches=n, total_ms=ms, mean_us=(1e3 * ms / n if n else 0.0)) for k, (n, ms) in prof.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    r = kernel_roofs(dom, shapes, kern[dom]["mean_us"], mixed, z_f32)
    # the committed counters were taken with the default FP64 Schur sums
    traffic = measured_traffic(args.workload, dom) if not args.fp32_accum else None
    common = dict(kernel=dom, traffic=traffic, flops_per_launch=r["flops_per_launch"],
                  bytes_per_launch=r["bytes_per_launch"], mean_us=r["mean_us"],
                  alu_TFLOPs=r["achieved_TFLOPs"], alu_frac=r["alu_frac"],
                  alu_frac_of_nonpacked_78_6=r["alu_frac_nonpacked"], hbm_GBs=r["achieved_GBs"],
                  hbm_frac=r["hbm_frac"])
    if r["alu_frac"] >= r["hbm_frac"]:
        roof = dict(bound="alu", achieved=r["achieved_TFLOPs"], peak=r["alu_peak"], unit="TFLOP/s",
                    frac=r["alu_frac"], **common)
    else:
        roof = dict(bound="hbm", achieved=r["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=r["hbm_frac"], **common)
    cp = copy_peak_gbs(dev)
    roof["copy_peak_GBs"] = cp
    roof["hbm_frac_of_copy_peak"] = r["achieved_GBs"] / cp
    streaming = {}
    for k in ("linearize", "update"):
        if kern[k]["launches"]:
            rk = kernel_roofs(k, shapes, kern[k]["mean_us"], mixed, z_f32)
            streaming[k] = {"mean_us": round(rk["mean_us"], 2), "GB/s": round(rk["achieved_GBs"], 1),
                            "hbm_frac": round(rk["hbm_frac"], 4), "frac_of_copy_peak": round(rk["achieved_GBs"] / cp, 4), "TFLOP/s": round(rk["achieved_TFLOPs"], 2),
                            "alu_frac": round(rk["alu_frac"], 4)}

    value = iters / el
    out = {
        "metric": METRIC,
        "value": value,
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
                   "observations": int(sum(s["N"] for s in shapes)),
                   "lm_iterations_per_step": iters // args.steps,
                   "schur_sums": "fp32" if (mixed and args.fp32_accum) else "fp64",
                   "points_per_tile_by_window_class": tuned},
        "graph_replay": {"value": giters / gel, "ms_per_step": 1e3 * gel / args.steps,
                         "note": "the timed steps repeated with each LM step replayed from its HIP graph "
                                 "(value above: kernels launched one by one between HIP events)"},
        "roofline": roof,
        "streaming_kernels": streaming,
        "kernels_us_mean": {k: round(v["mean_us"], 2) for k, v in kern.items() if v["launches"]},
    }

    if spec["compare_plain"] and not args.no_plain:
        # the same windows, one plain FP64 lba_solve call per window
        pctx = lba.Context(device=0, precision="fp64")
        solvers = [lba.Solver(pctx, lba.DeviceProblem(w, device=dev)) for w in windows]
        for s in solvers:
            s.run(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pit = 0
        for s in solvers:
            s.run(stream)
            pit += int(s.stats[0, 2] + s.stats[0, 3])
        torch.cuda.synchronize()
        pel = time.perf_counter() - t1
        out["plain_fp64_per_window"] = {"value": pit / pel, "unit": "window-LM-iterations/s",
                                        "seconds": pel, "windows": len(windows)}
        out["speedup_vs_plain_fp64"] = value / (pit / pel)
        print(f"bench: plain FP64 per-window pass {pel:.3f} s", file=sys.stderr, flush=True)
        del solvers

    if not args.no_cpu_baseline:
        cb, refs = cpu_baseline(windows, z_f32=z_f32)
        out["cpu_baseline"] = cb
        # parity spot check of the benchmarked solve: the oracle on the same (FP32-rounded
        # where the GPU read FP32) measurements, final cost and RMS reprojection difference
        from tests.parity import reprojection_rms_diff, round_z_f32
        T_out, X_out = solver.T_out.cpu().numpy(), solver.X_out.cpu().numpy()
        rel, px = [], []
        for i, r in refs.items():
            w = round_z_f32(windows[i]) if z_f32 else windows[i]
            k0, k1 = prob.kf_off[i], prob.kf_off[i + 1]
            p0, p1 = prob.pt_off[i], prob.pt_off[i + 1]
            rel.append(abs(solver.stats[i, 1] - r["stats"]["F_final"]) / abs(r["stats"]["F_final"]))
            px.append(reprojection_rms_diff(w, T_out[k0:k1], X_out[p0:p1], r["T"], r["X"], ~r["outlier"]))
        out["parity"] = {"windows_checked": len(rel), "final_cost_rel_max": float(max(rel)),
                         "rms_reprojection_diff_px_max": float(max(px)),
                         "oracle_inputs": "FP32-rounded measurements" if z_f32 else "FP64 measurements"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
