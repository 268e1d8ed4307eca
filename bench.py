"""Benchmark of the per-frame SIR step on one GPU.

Workload (default): a 1024x1024 uint8 video of 100 frames with a disk of radius
5 (intensity 228 on 100) moving (+1, -2) px per frame plus N(0, 2^2) noise;
N = 2^20 particles; transition (1, -2) + (5, 2) * N(0, 1); disk likelihood over
69 offsets; systematic resampling.  One "step" is one SIR step of one filter
on one frame (propagate, likelihood, maximum, weights, normalise + cumulative
distribution, systematic resampling, estimate) with the video resident in
device memory.

Prints one JSON line: FP16 particle-updates per second (the headline), the
other precisions on the same GPU, their track RMS against the FP64 track, the
roofline of the dominant kernel from HIP events over the timed region, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of one MI355X (vendor): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # lane-operation issue slots per second
PEAK_HBM = 8.0e12                      # bytes per second

# Algorithmic work of pass A per particle-update, in VALU lane-operation issue
# slots (a quarter-rate instruction costs 4), counted from the method's minimal
# instruction sequence per precision mode; the derivation is in the design doc.
PASS_A_SLOTS = {"f64": 330, "f32": 190, "f16": 186, "bf16": 192}
STATE_BYTES = {"f64": 32, "f32": 16, "f16": 8, "bf16": 8}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_mode(pf, torch, frames_dev, centres, w, dtype, steps, warmup, profile):
    T = frames_dev.shape[0]
    assert warmup + steps <= T - 1, "the timed steps must fit in one pass over the video"
    x0, y0 = centres[0]
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed)
    f = pf.Filter(p)
    t = 1
    for _ in range(warmup):
        f.step(frames_dev[t])
        t += 1
    if profile:
        pf.pf_profile_start(f.handle, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.step(frames_dev[t])
        t += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pf.pf_profile_read(f.handle) if profile else None
    f.close()
    return (t1 - t0), prof


def track(pf, frames_dev, centres, w, dtype, nsteps):
    """Free-running estimates over frames 1..nsteps (untimed)."""
    x0, y0 = centres[0]
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed)
    f = pf.Filter(p)
    est = [(x0, y0)]
    for t in range(1, nsteps + 1):
        f.step(frames_dev[t])
        est.append(f.estimate())
    f.close()
    return np.array(est)


def cpu_baseline(w, vid, budget_s):
    """The FP64 oracle (sequential C, one thread) on the first steps of the
    same video at the same N, as many steps as fit in about budget_s."""
    import oracle
    oracle.build(force=False)
    op = oracle.make_params(w.n_particles, w.width, w.height, radius=w.radius, drift=w.drift,
                            sigma=w.sigma, seed=w.filter_seed)
    x = np.full(w.n_particles, vid.centres[0][0])
    y = np.full(w.n_particles, vid.centres[0][1])
    t0 = time.perf_counter()
    steps = 0
    while steps < vid.frames.shape[0] - 1:
        out = oracle.step(op, steps + 1, vid.frames[steps + 1], x, y)
        x, y = out["x"], out["y"]
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=w.n_particles * steps / dt, unit="particle-updates/s", cores=1,
                kind="oracle",
                sample=f"first {steps} steps of {w.name} at N={w.n_particles}, FP64, 1 thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=80)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="disk1024_n1m")
    ap.add_argument("--modes", default="f16,f32,bf16,f64")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-track", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the filter step is single-GPU "
              "(sharding across GPUs is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2308_00763_amd as pf
    import pfsynth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    w = pfsynth.WORKLOADS[args.workload]
    log(f"[bench] generating {w.name}: {w.frames} frames {w.width}x{w.height}")
    vid = pfsynth.workload_video(w)
    frames_dev = torch.from_numpy(vid.frames).to("cuda:0")
    modes = args.modes.split(",")

    res = {}
    for dt in modes:
        log(f"[bench] timing {dt}: warmup {args.warmup}, steps {args.steps}")
        secs, prof = run_mode(pf, torch, frames_dev, vid.centres, w, dt, args.steps, args.warmup,
                              profile=True)
        a_ms, m_ms, c_ms, n = prof
        res[dt] = dict(seconds=secs, ms_per_step=1e3 * secs / args.steps,
                       updates_per_s=w.n_particles * args.steps / secs,
                       pass_a_us=1e3 * a_ms / n, combine_us=1e3 * m_ms / n, pass_c_us=1e3 * c_ms / n)
        log(f"[bench] {dt}: {res[dt]}")

    if not args.no_track and "f64" in modes:
        nsteps = args.warmup + args.steps
        ref = track(pf, frames_dev, vid.centres, w, "f64", nsteps)
        for dt in modes:
            est = ref if dt == "f64" else track(pf, frames_dev, vid.centres, w, dt, nsteps)
            res[dt]["track_rms_vs_f64_px"] = float(np.sqrt(np.mean(np.sum((est - ref) ** 2, axis=1))))
            res[dt]["track_rms_vs_truth_px"] = float(
                np.sqrt(np.mean(np.sum((est - vid.centres[:nsteps + 1]) ** 2, axis=1))))

    head = "f16" if "f16" in modes else modes[0]
    r = res[head]
    # dominant kernel: the longer of the two passes
    dom = "pass_a" if r["pass_a_us"] >= r["pass_c_us"] else "pass_c"
    a_s = r["pass_a_us"] * 1e-6
    if dom == "pass_a":
        achieved = PASS_A_SLOTS[head] * w.n_particles / a_s
        roof = dict(bound="alu", kernel="pass_a", achieved=achieved / 1e12, peak=PEAK_LANE_OPS / 1e12,
                    unit="Tlane-op/s", frac=achieved / PEAK_LANE_OPS, traffic=None,
                    kernel_us=r["pass_a_us"])
    else:
        c_s = r["pass_c_us"] * 1e-6
        byts = STATE_BYTES[head] * w.n_particles / 2  # pass C's share: read + write of positions
        achieved = byts / c_s
        roof = dict(bound="hbm", kernel="pass_c", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9,
                    unit="GB/s", frac=achieved / PEAK_HBM, traffic=None, kernel_us=r["pass_c_us"])

    out = {
        "metric": "particle-updates/sec FP16 vs FP64 at <=0.5px track error; p99 frame latency",
        "value": r["updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if head == "f16" else head,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.width}x{w.height} uint8, {w.frames} frames, disk r={w.radius}, "
                               f"noise sigma {w.noise_sigma}, N={w.n_particles}, one filter",
                   "n_particles": w.n_particles, "frame": [w.height, w.width], "radius": w.radius},
        "modes": res,
        "roofline": roof,
    }
    if "f64" in res:
        out["speedup_f16_vs_f64"] = res["f64"]["seconds"] / res.get("f16", res["f64"])["seconds"]
    if "f32" in res and "f16" in res:
        out["speedup_f16_vs_f32"] = res["f32"]["seconds"] / res["f16"]["seconds"]
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, vid, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
