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

# Algorithmic work of pass A per particle-update, in full-rate VALU
# instruction slots (a wave64 instruction issued every 4 cycles per SIMD is
# one slot per lane; measured on this GPU: transcendentals cost 2, 64-bit
# products and double operations 1.25), counted from the minimal instruction
# sequence of the method for radius 5: Philox4x32-10 65, uniforms 6,
# Box-Muller 12, propagation 3-5, pixel rounding 8, disk sum over the row
# prefixes 18 + 1, weight 5, maximum / prefix sum / estimate 4.  The double
# mode replaces the float uniforms, Box-Muller, propagation, rounding, weight
# and the likelihood division by their double versions.
PASS_A_SLOTS = {"f64": 277, "f32": 123, "f16": 122, "bf16": 124}  # at radius 5


def pass_a_slots(dtype, radius):
    """Algorithmic pass-A slots per update at disk radius r: the radius-5
    count with its 18 + 1 disk-sum slots replaced by 2 (2r - 1) + 1."""
    return PASS_A_SLOTS[dtype] - 19 + 2 * (2 * radius - 1) + 1
# Algorithmic bytes per update (spill-free): the particle's state read and
# its resampled state written, two coordinates of 8 / 4 / 2 / 2 bytes each way.
STATE_BYTES = {"f64": 32, "f32": 16, "f16": 8, "bf16": 8}
# Algorithmic VALU slots of resampling per update: the particle's end slot
# (one multiply-add, floor, conversion, compare), its first-slot mark, its
# share of the slot scan and the copy of its position.
RESAMPLE_SLOTS = 8
# Bytes per update that the two-pass step moves beyond the algorithmic ones:
# pass A writes the propagated state and the tile-local prefix sums, pass C
# reads them back.
SPILL_BYTES = {"f64": 2 * (16 + 8), "f32": 2 * (8 + 4), "f16": 2 * (4 + 4), "bf16": 2 * (4 + 4)}


def step_slots(dtype, radius):
    """Algorithmic VALU slots of one whole step per update."""
    return pass_a_slots(dtype, radius) + RESAMPLE_SLOTS


def step_bound_s(dtype, radius, n):
    """Roofline time of one step of n particles on the algorithmic work only:
    the larger of the VALU time of every step part (pass-A slots plus
    resampling) and the HBM time of the state read and written.  The spill of
    the propagated state and prefix sums between passes is not algorithmic
    work and is not counted."""
    return n * max(step_slots(dtype, radius) / PEAK_LANE_OPS, STATE_BYTES[dtype] / PEAK_HBM)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "step_traffic_f16_disk1024_n1m.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2308_00763_amd", "csrc", f)
                  for f in ("kernels.hip", "philox.hpp", "wave.hpp", "pf_internal.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_values():
    """Machine-readable values of the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return vals


def measured_traffic(kernel, dtype):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's counts), if
    it was taken on the current kernel sources for this mode (else None)."""
    vals = _traffic_values()
    if vals is None or vals.get("dtype") != dtype or f"{kernel}_fetch_kib" not in vals:
        return None
    fetch = float(vals[f"{kernel}_fetch_kib"]) * 1024 * float(vals["fetch_scale"])
    write = float(vals[f"{kernel}_write_kib"]) * 1024 * float(vals["write_scale"])
    return fetch + write


def measured_step_traffic(dtype):
    """HBM bytes of one whole step (every kernel of the step) from the same
    summary, or None."""
    vals = _traffic_values()
    if vals is None or vals.get("dtype") != dtype:
        return None
    ks = [k.strip() for k in vals.get("kernels", "").split(",") if k.strip()]
    parts = [measured_traffic(k, dtype) for k in ks]
    return sum(parts) if parts and None not in parts else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_mode(pf, torch, frames_dev, centres, w, dtype, steps, warmup, profile, **variant):
    """Time `steps` SIR steps after `warmup` (a fresh filter each call).

    The timed loop calls the C ABI directly with precomputed frame pointers,
    so the host adds as little as possible between launches.  With profile=True
    the same loop also records HIP events around every kernel (on the filter's
    stream); event records between kernels lengthen the step, so the headline
    time comes from a run without them."""
    import ctypes
    T = frames_dev.shape[0]
    assert warmup + steps <= T - 1, "the timed steps must fit in one pass over the video"
    x0, y0 = centres[0]
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed, **variant)
    f = pf.Filter(p)
    lib = pf.lib()
    pitch = int(frames_dev.stride(1))
    base = int(frames_dev.data_ptr())
    fstride = int(frames_dev.stride(0))
    ptrs = [ctypes.c_void_p(base + t * fstride) for t in range(T)]
    step = lib.pf_step
    h = f.handle
    for t in range(1, warmup + 1):
        if step(h, ptrs[t], pitch):
            raise pf.PfError(-1, pf.pf_last_error())
    if profile:
        pf.pf_profile_start(h, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        step(h, ptrs[t], pitch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pf.pf_profile_read(h) if profile else None
    f.close()
    return (t1 - t0), prof


def warm_gpu(pf, torch, frames_dev, centres, w, dtype, seconds, **variant):
    """Run the workload's steps untimed for about `seconds` (a fresh filter
    for every pass over the video, so every step is a tracking step like the
    timed ones) so that the GPU's clocks have ramped up before the first
    timed mode (the first mode timed in a fresh process otherwise runs its
    pass A about 12 % slower than later modes).  Returns the steps run."""
    import ctypes
    T = frames_dev.shape[0]
    x0, y0 = centres[0]
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed, **variant)
    lib = pf.lib()
    pitch = int(frames_dev.stride(1))
    base = int(frames_dev.data_ptr())
    fstride = int(frames_dev.stride(0))
    ptrs = [ctypes.c_void_p(base + t * fstride) for t in range(T)]
    n = 0
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        f = pf.Filter(p)
        for t in range(1, T):
            n += 1
            if lib.pf_step(f.handle, ptrs[t], pitch):
                raise pf.PfError(-1, pf.pf_last_error())
        torch.cuda.synchronize()
        f.close()
    return n


def track(pf, frames_dev, centres, w, dtype, nsteps, **variant):
    """Free-running estimates over frames 1..nsteps (untimed)."""
    x0, y0 = centres[0]
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed, **variant)
    f = pf.Filter(p)
    est = [(x0, y0)]
    for t in range(1, nsteps + 1):
        f.step(frames_dev[t])
        est.append(f.estimate())
    f.close()
    return np.array(est)


def run_fleet(pf, torch, pfsynth, n_streams, side, frames, steps, warmup, dtype="f16"):
    """The stream fleet: n_streams independent filters (N log-uniform in
    [256, 65536]) on their own side x side videos, drawn on the device and
    resident before timing; one pf_batch_step per frame index."""
    import ctypes
    assert warmup + steps <= frames - 2
    streams = pfsynth.stream_mix(n_streams, side=side, frames=frames)
    log(f"[bench] fleet: drawing {frames} frames of {n_streams} streams ({side}x{side}) on the device")
    vids = torch.stack([pfsynth.render_fleet_torch(streams, t, side, 5, "cuda:0", seed=4_000_000)
                        for t in range(frames)])  # (T, n, side, side)
    params = [pf.make_params(s.n_particles, side, side, dtype, radius=5, x0=s.start[0],
                             y0=s.start[1], drift=s.velocity, seed=0, stream_id=s.stream_id)
              for s in streams]
    side_stream = torch.cuda.Stream()  # a stream that can be captured
    b = pf.Batch(params, stream=side_stream)
    base = int(vids.data_ptr())
    fstride, sstride = int(vids.stride(0)), int(vids.stride(1))
    ptrs = [np.array([base + t * fstride + k * sstride for k in range(n_streams)], dtype=np.uint64)
            for t in range(frames)]
    pitches = np.full(n_streams, int(vids.stride(2)), dtype=np.int64)
    step = pf.lib().pf_batch_step
    pp = ctypes.c_void_p(pitches.ctypes.data)
    h = b.handle
    for t in range(1, warmup + 1):
        if step(h, ctypes.c_void_p(ptrs[t].ctypes.data), pp, None):
            raise pf.PfError(-1, pf.pf_last_error())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        step(h, ctypes.c_void_p(ptrs[t].ctypes.data), pp, None)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    est = b.estimates()
    t_end = warmup + steps
    truth = np.array([[s.start[0] + s.velocity[0] * t_end, s.start[1] + s.velocity[1] * t_end]
                      for s in streams])
    err = np.hypot(*(est - truth).T)
    # the same step captured in a HIP graph and replayed (on the next frame
    # index's frames, the same ones at every replay)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side_stream):
        if step(h, ctypes.c_void_p(ptrs[t_end + 1].ctypes.data), pp, None):
            raise pf.PfError(-1, pf.pf_last_error())
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    gsecs = time.perf_counter() - t0
    assert np.all(np.isfinite(b.estimates()))
    del g
    b.close()
    total = sum(p.n_particles for p in params)
    return dict(workload=f"{n_streams} streams, {side}x{side} uint8 video each (drawn on the device), "
                         f"{frames} frames, disk r=5, noise sigma U[2,6], velocity in {{-3..3}}^2, "
                         f"N log-uniform in [256, 65536]",
                dtype=dtype, filters=n_streams, particles=total, steps=steps, warmup=warmup,
                ms_per_step=1e3 * secs / steps, updates_per_s=total * steps / secs,
                step_roofline_frac=step_bound_s(dtype, 5, total) / (secs / steps),
                graph_ms_per_step=1e3 * gsecs / steps,
                final_error_median_px=float(np.median(err)),
                final_error_p99_px=float(np.percentile(err, 99)))


SERVE_SIDES = (64, 128, 256, 512, 1024)
SERVE_BANK_T = 560


def _serving_bank(torch, pfsynth, rng):
    """Device-resident bank of bouncing-disk videos: four per frame side,
    560 frames each, noise sigma ~ U[2, 6], velocity in {-3..3}^2."""
    log("[bench] serving: drawing the video bank on the device")
    bank = {}
    for side in SERVE_SIDES:
        for j in range(4):
            v = (int(rng.integers(-3, 4)), int(rng.integers(-3, 4)))
            start = (int(rng.integers(5, side - 5)), int(rng.integers(5, side - 5)))
            cen = pfsynth.trajectory(SERVE_BANK_T, start, v, side, side, 5, bounce=True)
            sig = float(rng.uniform(2.0, 6.0))
            bank[(side, j)] = (cen, pfsynth.render_video_torch(cen, side, 5, sig, "cuda:0",
                                                                seed=7_000 + 10 * side + j))
    return bank


SERVE_HANDLES = 2048  # batch members per precision: the most streams served at once


def _serving_pools(hbm_gb, admission="bytes"):
    """The serving backend for HBM budgets hbm_gb = (FP16 GiB, FP32 GiB):
    admission by bytes (every stream gets exactly its workspace from the
    budget) or by power-of-two slot classes sized from the budget."""
    from paper_2308_00763_amd.serve import GpuByteBackend, GpuPoolBackend, plan_pool, slot_classes
    if admission == "bytes":
        budgets = {"f16": int(hbm_gb[0] * 2**30), "f32": int(hbm_gb[1] * 2**30)}
        log(f"[bench] serving: byte budgets {budgets}, {SERVE_HANDLES} handles per precision")
        return GpuByteBackend(budgets, {"f16": SERVE_HANDLES, "f32": SERVE_HANDLES})
    caps = slot_classes(1000, 1_000_000)
    pools = {"f16": plan_pool(int(hbm_gb[0] * 2**30), "f16", caps),
             "f32": plan_pool(int(hbm_gb[1] * 2**30), "f32", caps)}
    log(f"[bench] serving: pools {pools}")
    return GpuPoolBackend(pools)


def _serving_request(pf, rng, bank, sid, arrival, fps, frames=None):
    """One stream of the serving mix: frames ~ U{20..500} (or `frames`), side
    ~ U{64, ..., 1024}, N = round(exp(U(ln 1e3, ln 1e6))), FP16 or FP32 with
    probability 1/2, from a random bank video at a random start frame."""
    from paper_2308_00763_amd.serve import FrameSeq, StreamRequest
    frames = int(rng.integers(20, 501)) if frames is None else frames
    side = int(rng.choice(SERVE_SIDES))
    j = int(rng.integers(0, 4))
    cen, vid = bank[(side, j)]
    o = int(rng.integers(0, SERVE_BANK_T - frames + 1))
    n = int(round(float(np.exp(rng.uniform(np.log(1e3), np.log(1e6))))))
    dtype = "f16" if rng.random() < 0.5 else "f32"
    d = cen[o + 1] - cen[o]
    p = pf.make_params(n, side, side, dtype, x0=cen[o][0], y0=cen[o][1], drift=(d[0], d[1]),
                       seed=5, stream_id=sid)
    base, fst, pitch = int(vid.data_ptr()), int(vid.stride(0)), int(vid.stride(1))
    return StreamRequest(sid, arrival, p, frames, fps, FrameSeq(base + o * fst, fst, pitch))


def run_serving(pf, torch, pfsynth, seconds, warmup_s, rate=200.0, fps=30.0, hbm_gb=(6.0, 12.0),
                admission="bytes"):
    """Continuous batching of arriving streams: Poisson arrivals at `rate`
    streams/s (PCG64(5)); per stream frames ~ U{20..500} at `fps`, side ~
    U{64, 128, 256, 512, 1024}, N = round(exp(U(ln 1e3, ln 1e6))), FP16 or FP32
    with probability 1/2, disk r = 5, noise sigma ~ U[2, 6], velocity in
    {-3..3}^2 with specular bounce.  Frames come from a device-resident bank of
    bouncing-disk videos (four per side, 560 frames) at a random start frame.
    Latency is frame arrival to estimate ready, over frames arriving after
    `warmup_s`."""
    from paper_2308_00763_amd.serve import Scheduler
    rng = np.random.Generator(np.random.PCG64(5))
    bank = _serving_bank(torch, pfsynth, rng)
    be = _serving_pools(hbm_gb, admission)
    sched = Scheduler(be, stall_timeout=5.0)
    total = warmup_s + seconds
    t = 0.0
    sid = 0
    t_base = time.perf_counter() + 1.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > total:
            break
        sched.submit(_serving_request(pf, rng, bank, sid, t_base + t, fps))
        sid += 1
    log(f"[bench] serving: {sid} streams over {total:.0f} s; running")
    while time.perf_counter() < t_base:
        time.sleep(0.01)
    n_warm = None
    last = time.perf_counter()
    while not sched.idle() and time.perf_counter() < t_base + total + 30.0:
        if sched.tick() == 0:
            time.sleep(0.0002)
        now = time.perf_counter()
        if n_warm is None and now >= t_base + warmup_s:
            n_warm = len(sched.latencies)
            u_warm = sched.updates
            t_warm = now
        if now - last > 5.0:
            log(f"[bench] serving: t={now - t_base:.0f} s, live {len(sched.live)}, queued {len(sched.queue)}, "
                f"frames {len(sched.latencies)}")
            last = now
        if now >= t_base + total:
            break
    t_end = time.perf_counter()
    summ = sched.summary(since_latency=n_warm or 0)
    summ.update(workload=f"Poisson arrivals at {rate:g} streams/s for {seconds:g} s after {warmup_s:g} s warm-up; "
                         f"per stream U{{20..500}} frames at {fps:g} fps, side U{{64..1024}}, "
                         f"N log-uniform [1e3, 1e6], FP16 or FP32, r=5, bounce",
                updates_per_s=(sched.updates - (u_warm if n_warm is not None else 0)) /
                              max(t_end - (t_warm if n_warm is not None else t_base), 1e-9),
                live_at_end=len(sched.live), queued_at_end=len(sched.queue),
                pool_bytes=be.pool_bytes, streams_submitted=sid, admission=admission)
    be.close()
    return summ


def run_serving_closed(pf, torch, pfsynth, seconds, n_streams=1770, hbm_gb=(6.0, 12.0), admission="bytes"):
    """Closed-loop serving capacity: a constant population of n_streams
    streams of the serving mix (500 frames each; a finished stream is
    replaced at once), every frame already waiting (a frame rate far above
    what is served), so every tick steps every live stream; ticks, frames and
    particle-updates per second over `seconds`."""
    from paper_2308_00763_amd.serve import Scheduler
    rng = np.random.Generator(np.random.PCG64(6))
    bank = _serving_bank(torch, pfsynth, rng)
    be = _serving_pools(hbm_gb, admission)
    sched = Scheduler(be, stall_timeout=60.0)
    sid = 0

    def top_up():
        # streams in the population: admitted, waiting for a slot, or submitted
        # and not yet arrived (a rejected submission ends the top-up)
        nonlocal sid
        now = time.perf_counter()
        while len(sched.live) + len(sched.queue) + len(sched.pending) < n_streams:
            ok = sched.submit(_serving_request(pf, rng, bank, sid, now, 1.0e6, frames=500))
            sid += 1
            if not ok:
                break

    top_up()
    for _ in range(20):  # warm-up ticks
        sched.tick()
        top_up()
    ticks = 0
    f0, u0, s0 = len(sched.latencies), sched.updates, sched.step_seconds
    t_start = time.perf_counter()
    while time.perf_counter() < t_start + seconds:
        sched.tick()
        top_up()
        ticks += 1
    dt = time.perf_counter() - t_start
    out = dict(workload=f"{n_streams} live streams of the serving mix, 500 frames each, a finished stream "
                        f"replaced at once, every frame waiting", seconds=dt, ticks_per_s=ticks / dt,
               frames_per_s=(len(sched.latencies) - f0) / dt, updates_per_s=(sched.updates - u0) / dt,
               # the backend's share of a tick (the batched steps and the
               # estimates' read-back, which waits for them); the rest is
               # the scheduler's own per-stream work on the host
               backend_ms_per_tick=1e3 * (sched.step_seconds - s0) / max(ticks, 1),
               ms_per_tick=1e3 * dt / max(ticks, 1), streams_submitted=sid, live_at_end=len(sched.live), queued_at_end=len(sched.queue))
    be.close()
    return out


ABLATION = [
    ("optimised", {}),
    ("naive likelihood (every disk pixel from the frame)", dict(naive_likelihood=True)),
    ("naive resampling, 64 threads", dict(naive_resample=True, threads_c=64)),
    ("naive resampling, 128 threads", dict(naive_resample=True, threads_c=128)),
    ("naive resampling, 256 threads", dict(naive_resample=True, threads_c=256)),
    ("naive resampling, 512 threads", dict(naive_resample=True, threads_c=512)),
    ("naive resampling, 1024 threads", dict(naive_resample=True, threads_c=1024)),
    ("naive likelihood + resampling, 128 threads",
     dict(naive_likelihood=True, naive_resample=True, threads_c=128)),
    ("unpacked half propagation (FP16 only)", dict(naive_half=True)),
    ("naive half step: unpacked half + division per particle in the resampler (FP16 only)",
     dict(naive_half=True, naive_resample=True)),
    ("pass A 128 threads (8 particles each)", dict(threads_a=128)),
    ("pass A 256 threads (4 particles each)", dict(threads_a=256)),
    ("pass A 512 threads (2 particles each)", dict(threads_a=512)),
    ("pass C 64 threads", dict(threads_c=64)),
    ("pass C 128 threads", dict(threads_c=128)),
    ("pass C 256 threads", dict(threads_c=256)),
    ("pass C 512 threads", dict(threads_c=512)),
    ("pass C 1024 threads", dict(threads_c=1024)),
]


def run_ablation(pf, torch, frames_dev, centres, w, steps, warmup, dtypes=("f16", "f64")):
    """The straightforward step against the optimised one, and workgroup
    sizes, at the headline workload: ms per step and per-pass times."""
    res = {}
    for dt in dtypes:
        rows = {}
        for name, var in ABLATION:
            if var.get("naive_half") and dt != "f16":
                continue
            secs, _ = run_mode(pf, torch, frames_dev, centres, w, dt, steps, warmup, False, **var)
            _, prof = run_mode(pf, torch, frames_dev, centres, w, dt, steps, warmup, True, **var)
            a_ms, m_ms, c_ms, n = prof
            # resample_us 0: an FP64 filter at the default sizes resamples in
            # the next step's pass A (deferred resampling)
            rows[name] = dict(ms_per_step=1e3 * secs / steps, pass_a_us=1e3 * a_ms / n,
                              combine_us=1e3 * m_ms / n, resample_us=1e3 * c_ms / n,
                              resample_in_pass_a=c_ms == 0.0)
        res[dt] = rows
    return res


def run_resamplers(pf, torch, frames_dev, centres, w, steps, warmup, dtypes=("f16", "f64")):
    """Systematic resampling against Metropolis (B = 8, 32, 128) at the
    headline size, and against Gumbel-max multinomial resampling at N = 65536
    (its limit): ms per step, resampling kernel time, and the RMS distance of
    the free-running track to the ground truth over the timed frames."""
    import dataclasses
    nsteps = warmup + steps
    cases = [(w, "systematic", {}), (w, "metropolis B=8", dict(metropolis_steps=8)),
             (w, "metropolis B=32", dict(metropolis_steps=32)),
             (w, "metropolis B=128", dict(metropolis_steps=128)),
             (w, "rejection, at most 4096 trials", dict(rejection_trials=4096))]
    w64 = dataclasses.replace(w, n_particles=65536, name=w.name + "_n65536")
    cases += [(w64, "systematic", {}), (w64, "gumbel-max", dict(gumbel_max=True))]
    res = {}
    for dt in dtypes:
        rows = []
        for wl, name, var in cases:
            secs, _ = run_mode(pf, torch, frames_dev, centres, wl, dt, steps, warmup, False, **var)
            _, prof = run_mode(pf, torch, frames_dev, centres, wl, dt, steps, warmup, True, **var)
            est = track(pf, frames_dev, centres, wl, dt, nsteps, **var)
            rms = float(np.sqrt(np.mean(np.sum((est - centres[:nsteps + 1]) ** 2, axis=1))))
            rows.append(dict(resampler=name, n_particles=wl.n_particles, ms_per_step=1e3 * secs / steps,
                             resample_us=1e3 * prof[2] / prof[3], resample_in_pass_a=prof[2] == 0.0,
                             track_rms_vs_truth_px=rms))
        res[dt] = rows
    return res


RESAMPLER_CASES = [("systematic", {}), ("metropolis B=8", dict(metropolis_steps=8)),
                   ("metropolis B=32", dict(metropolis_steps=32)),
                   ("metropolis B=128", dict(metropolis_steps=128)),
                   ("rejection, at most 4096 trials", dict(rejection_trials=4096))]


def run_resampler_bias(pf, torch, pfsynth, runs=8, steps=10, dtype="f16"):
    """Bias and speed of the resamplers at 2^24 particles (512x512, radius 8,
    noise sigma 8).  Speed: ms per step and resampling kernel time on the
    video.  Bias: a cloud of particles around the object (normal offsets of
    3 px per axis, seeded) is frozen (no drift, no noise) and resampled
    `runs` times with fresh random streams, so the normalised weights w are
    the same in every run; offspring counts averaged over the runs are
    compared with N w, per pixel cell (particles in one cell share their
    weight): TV = 1/2 sum over cells |mean offspring share - weight share|.
    An unbiased multinomial resampler's TV from its noise alone is about
    1/2 sum sqrt(2 W (1 - W) / (pi N runs)) over the cells' weights W (the
    "multinomial_floor"); systematic resampling's counts vary less, a biased
    resampler's TV stays above the floor however many runs."""
    wl = pfsynth.WORKLOADS["disk512_r8_n16m"]
    n = wl.n_particles
    vid = pfsynth.workload_video(wl, frames=steps + 12)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    cx, cy = vid.centres[4]
    rng = np.random.Generator(np.random.PCG64(11))
    xs = cx + 3.0 * rng.standard_normal(n)
    ys = cy + 3.0 * rng.standard_normal(n)
    cell = (np.floor(ys + 0.5).astype(np.int64) * 4096 + np.floor(xs + 0.5).astype(np.int64))
    _, cell_id = np.unique(cell, return_inverse=True)
    out = {"workload": f"{wl.name}: N={n}, radius {wl.radius}, noise sigma {wl.noise_sigma}, {dtype}; "
                       f"frozen cloud of N(0, 3^2) offsets around the object for the bias",
           "runs": runs, "rows": []}
    floor = None
    for name, var in RESAMPLER_CASES:
        log(f"[bench] resampler bias: {name}")
        secs, _ = run_mode(pf, torch, fr, vid.centres, wl, dtype, steps, 1, False, **var)
        _, prof = run_mode(pf, torch, fr, vid.centres, wl, dtype, steps, 1, True, **var)
        g = pf.Filter(pf.make_params(n, wl.width, wl.height, dtype, radius=wl.radius, x0=x0, y0=y0,
                                     drift=(0.0, 0.0), sigma=(0.0, 0.0), seed=wl.filter_seed,
                                     diagnostics=True, **var))
        counts = np.zeros(n)
        w = None
        for r in range(runs):
            g.load(xs, ys, 3 + r)
            g.step(fr[4])
            e = g.export()
            counts += np.bincount(e["anc"], minlength=n)
            w = e["w"] if w is None else w
        g.close()
        W = np.bincount(cell_id, weights=w)
        share = np.bincount(cell_id, weights=counts) / (n * runs)
        tv = 0.5 * float(np.sum(np.abs(share - W)))
        if floor is None:
            floor = 0.5 * float(np.sum(np.sqrt(2 * W * (1 - W) / (np.pi * n * runs))))
        out["rows"].append(dict(resampler=name, ms_per_step=1e3 * secs / steps,
                                resample_us=1e3 * prof[2] / prof[3], cell_tv=tv))
    out["multinomial_floor"] = floor
    out["cells"] = int(cell_id.max() + 1)
    return out


# The paper's FP16 speedups (whole application, 32k and 64k particles, on
# V100, A100, A40 and T4): context for this GPU's ratios, not a target.
PAPER_SPEEDUPS = {"fp16_vs_fp32": "1.5-2x", "fp16_vs_fp64": "2.5-4.6x",
                  "hardware": "V100, A100, A40, T4", "particles": "32768 and 65536"}


def run_paper_sizes(pf, torch, frames_dev, centres, w, steps, warmup):
    """FP16, FP32 and FP64 steps at the paper's particle counts on the
    headline video, with the FP16 speedups the paper reports for them."""
    import dataclasses
    out = {"paper": PAPER_SPEEDUPS}
    for n in (32768, 65536):
        wl = dataclasses.replace(w, n_particles=n, name=f"{w.name}_n{n}")
        ms = {}
        for dt in ("f16", "f32", "f64"):
            secs, _ = run_mode(pf, torch, frames_dev, centres, wl, dt, steps, warmup, False)
            ms[dt] = 1e3 * secs / steps
        out[str(n)] = dict(ms_per_step=ms, fp16_vs_fp32=ms["f32"] / ms["f16"], fp16_vs_fp64=ms["f64"] / ms["f16"])
    return out


def run_accuracy(pf, torch, pfsynth, modes):
    """The paper's accuracy video (512x512, 100 frames, bounce off y = 0,
    128 particles): per mode the RMS distance of the free-running estimates to
    the ground truth, the largest distance to the FP64 estimates, and the
    share of frames whose rounded estimate equals the FP64 one."""
    w = pfsynth.WORKLOADS["bounce512_n128"]
    vid = pfsynth.workload_video(w, bounce=True)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    tr = {dt: track(pf, fr, vid.centres, w, dt, w.frames - 1) for dt in modes}
    res = {}
    for dt, e in tr.items():
        r = dict(rms_vs_truth_px=float(np.sqrt(np.mean(np.sum((e - vid.centres) ** 2, axis=1)))),
                 max_vs_truth_px=float(np.max(np.hypot(*(e - vid.centres).T))))
        if "f64" in tr:
            rms = float(np.sqrt(np.mean(np.sum((e - tr["f64"]) ** 2, axis=1))))
            r["rms_vs_f64_px"] = rms
            r["max_vs_f64_px"] = float(np.max(np.hypot(*(e - tr["f64"]).T)))
            r["rounded_equal_f64"] = float(np.mean(np.all(np.rint(e) == np.rint(tr["f64"]), axis=1)))
            # the accuracy bound of the reduced modes: RMS distance to the FP64
            # track at most 0.5 px (False: the mode misses it on this video)
            r["within_0p5px_of_f64"] = rms <= 0.5
        res[dt] = r
    return dict(workload=f"{w.name}: {w.width}x{w.height}, {w.frames} frames, bounce off y = 0 at frame 47, "
                         f"N={w.n_particles}", modes=res)


def run_large(pf, torch, pfsynth, args, modes):
    """The second single-filter workload (default 2^24 particles, r = 8) in
    every mode, with each mode's track RMS against FP64."""
    wl = pfsynth.WORKLOADS[args.large]
    log(f"[bench] generating {wl.name}: {wl.frames} frames {wl.width}x{wl.height}")
    vl = pfsynth.workload_video(wl)
    fl = torch.from_numpy(vl.frames).to("cuda:0")
    ls, lw = min(args.steps, wl.frames - 6), 5
    if args.gpu_warmup_s > 0:  # the heavier workload ramps the clocks again
        warm_gpu(pf, torch, fl, vl.centres, wl, modes[0], args.gpu_warmup_s)
    lres = {}
    for dt in modes:
        secs, _ = run_mode(pf, torch, fl, vl.centres, wl, dt, ls, lw, profile=False)
        _, prof = run_mode(pf, torch, fl, vl.centres, wl, dt, ls, lw, profile=True)
        a_us = 1e3 * prof[0] / prof[3]
        lres[dt] = dict(ms_per_step=1e3 * secs / ls, updates_per_s=wl.n_particles * ls / secs,
                        step_roofline_frac=step_bound_s(dt, wl.radius, wl.n_particles) / (secs / ls),
                        pass_a_us=a_us, combine_us=1e3 * prof[1] / prof[3],
                        pass_c_us=1e3 * prof[2] / prof[3],
                        pass_a_roofline_frac=pass_a_slots(dt, wl.radius) * wl.n_particles
                        / (a_us * 1e-6) / PEAK_LANE_OPS)
    if not args.no_track and "f64" in modes:
        ref = track(pf, fl, vl.centres, wl, "f64", wl.frames - 1)
        for dt in modes:
            est = ref if dt == "f64" else track(pf, fl, vl.centres, wl, dt, wl.frames - 1)
            lres[dt]["track_rms_vs_f64_px"] = float(np.sqrt(np.mean(np.sum((est - ref) ** 2, axis=1))))
    return dict(workload=f"{wl.name}: {wl.width}x{wl.height}, {wl.frames} frames, disk r={wl.radius}, "
                         f"noise sigma {wl.noise_sigma}, N={wl.n_particles}, one filter",
                steps=ls, warmup=lw, modes=lres)


def _oracle_rate(pfsynth, w, vid, budget_s, max_steps=None, repeat=False):
    """Particle-updates/s of the oracle's OpenMP timing build on one filter
    of workload w over the frames of vid, stepping until about budget_s
    (whole passes over the video when `repeat`)."""
    import oracle
    op = oracle.make_params(w.n_particles, w.width, w.height, radius=w.radius, drift=w.drift,
                            sigma=w.sigma, seed=w.filter_seed)
    T = vid.frames.shape[0]
    last = T - 1 if max_steps is None else min(T - 1, max_steps)
    steps = 0
    t0 = time.perf_counter()
    while True:
        st = oracle.OmpStepper(op, np.full(w.n_particles, vid.centres[0][0]),
                               np.full(w.n_particles, vid.centres[0][1]))
        for t in range(1, last + 1):
            st.step(t, vid.frames[t])
            steps += 1
            if not repeat and time.perf_counter() - t0 > budget_s:
                break
        if not repeat or time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return w.n_particles * steps / dt, steps, st.threads


def cpu_baseline(w, vid, budget_s, pfsynth):
    """The FP64 oracle timed on the host's cores: its OpenMP timing build
    (the sequential oracle's per-particle functions, per-thread partial sums
    and a two-pass parallel scan), as many threads as OpenMP is given, on a
    bounded sample of each single-GPU workload: the headline video
    (`value`), the 128 px parity video, the 2^24-particle video and a 5 %
    sample of the 4096-stream fleet.  About budget_s seconds per workload."""
    import oracle
    oracle.build(force=False)
    per = {}
    rate, steps, thr = _oracle_rate(pfsynth, w, vid, budget_s)
    per[w.name] = dict(value=rate, sample=f"first {steps} steps at N={w.n_particles}")
    w1 = pfsynth.WORKLOADS["disk128_n1000"]
    r1, s1, _ = _oracle_rate(pfsynth, w1, pfsynth.workload_video(w1), budget_s / 4, repeat=True)
    per[w1.name] = dict(value=r1, sample=f"{s1} steps (whole 9-step runs, repeated) at N=1000")
    w3 = pfsynth.WORKLOADS["disk512_r8_n16m"]
    r3, s3, _ = _oracle_rate(pfsynth, w3, pfsynth.workload_video(w3, frames=6), budget_s, max_steps=5)
    per[w3.name] = dict(value=r3, sample=f"first {s3} steps at N={w3.n_particles}, radius 8")
    # the fleet: every 20th of the 4096 streams (205 filters), 10 steps each
    streams = pfsynth.stream_mix(4096, side=256, frames=50)[::20]
    upd = 0
    t0 = time.perf_counter()
    for s in streams:
        v = pfsynth.stream_video(s, 256, 11)
        p = oracle.make_params(s.n_particles, 256, 256, radius=5, drift=s.velocity, seed=0,
                               stream_id=s.stream_id)
        st = oracle.OmpStepper(p, np.full(s.n_particles, float(s.start[0])),
                               np.full(s.n_particles, float(s.start[1])))
        for t in range(1, 11):
            st.step(t, v.frames[t])
        upd += 10 * s.n_particles
    r4 = upd / (time.perf_counter() - t0)
    per["fleet4096_256px"] = dict(value=r4, sample=f"every 20th of the 4096 streams ({len(streams)} filters, "
                                                   f"{upd} updates), first 10 steps each, one filter at a time")
    return dict(value=rate, unit="particle-updates/s", cores=thr, kind="oracle",
                sample=f"first {steps} steps of {w.name} at N={w.n_particles}, FP64, OpenMP timing build "
                       f"of the oracle on {thr} threads (host CPUs visible: {os.cpu_count()})",
                per_workload=per)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=80)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="disk1024_n1m")
    ap.add_argument("--modes", default="f16,f32,bf16,f64")
    ap.add_argument("--cpu-budget", type=float, default=6.0,
                    help="seconds of oracle timing per workload of the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-track", action="store_true")
    ap.add_argument("--large", default="disk512_r8_n16m",
                    help="second single-filter workload timed in every mode ('none' to skip)")
    ap.add_argument("--fleet", type=int, default=4096, metavar="STREAMS",
                    help="streams of the batched fleet workload (0 to skip)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the naive-vs-optimised and workgroup-size runs")
    ap.add_argument("--gpu-warmup-s", type=float, default=1.0,
                    help="seconds of untimed steps before the first timed mode (clock ramp-up)")
    ap.add_argument("--serve-admission", choices=("bytes", "classes"), default="bytes",
                    help="serving admission: by bytes from the HBM budget, or by power-of-two slot classes")
    ap.add_argument("--serve-hbm-gb", default="6,12", metavar="F16,F32",
                    help="serving HBM budgets in GiB for the FP16 and FP32 streams")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured seconds of the serving workload after a 10 s warm-up (0 to skip)")
    ap.add_argument("--variant", default="", metavar="KEY=VAL,...",
                    help="implementation variant for the timed modes, as make_params keywords "
                         "(e.g. naive_half=1,naive_resample=1)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (five times), "
                         "to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the filter step is single-GPU "
              "(sharding a filter across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2308_00763_amd as pf
    import pfsynth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 5}), flush=True)
        return
    w = pfsynth.WORKLOADS[args.workload]
    log(f"[bench] generating {w.name}: {w.frames} frames {w.width}x{w.height}")
    vid = pfsynth.workload_video(w)
    frames_dev = torch.from_numpy(vid.frames).to("cuda:0")
    modes = args.modes.split(",")
    variant = {}
    for kv in filter(None, args.variant.split(",")):
        key, val = kv.split("=")
        variant[key] = int(val)

    if args.gpu_warmup_s > 0:
        nw = warm_gpu(pf, torch, frames_dev, vid.centres, w, modes[0], args.gpu_warmup_s, **variant)
        log(f"[bench] GPU warm-up: {nw} untimed {modes[0]} steps in {args.gpu_warmup_s:g} s")
    res = {}
    for dt in modes:
        log(f"[bench] timing {dt}: warmup {args.warmup}, steps {args.steps}")
        secs, _ = run_mode(pf, torch, frames_dev, vid.centres, w, dt, args.steps, args.warmup,
                           profile=False, **variant)
        # the same steps again, with HIP events around every kernel
        psecs, prof = run_mode(pf, torch, frames_dev, vid.centres, w, dt, args.steps, args.warmup,
                               profile=True, **variant)
        a_ms, m_ms, c_ms, n = prof
        res[dt] = dict(seconds=secs, ms_per_step=1e3 * secs / args.steps,
                       updates_per_s=w.n_particles * args.steps / secs,
                       step_roofline_frac=step_bound_s(dt, w.radius, w.n_particles) / (secs / args.steps),
                       pass_a_us=1e3 * a_ms / n, combine_us=1e3 * m_ms / n, pass_c_us=1e3 * c_ms / n,
                       ms_per_step_with_events=1e3 * psecs / args.steps)
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
    if dom == "pass_a":
        a_s = r["pass_a_us"] * 1e-6
        achieved = pass_a_slots(head, w.radius) * w.n_particles / a_s
        roof = dict(bound="alu", kernel="pass_a", achieved=achieved / 1e12, peak=PEAK_LANE_OPS / 1e12,
                    unit="Tlane-op/s", frac=achieved / PEAK_LANE_OPS,
                    traffic=measured_traffic("pass_a", head) if w.name == "disk1024_n1m" else None,
                    kernel_us=r["pass_a_us"],
                    work_per_update=pass_a_slots(head, w.radius), work_unit="VALU lane slots")
    else:
        # pass C's algorithmic bytes: the resampled state it writes
        c_s = r["pass_c_us"] * 1e-6
        achieved = STATE_BYTES[head] // 2 * w.n_particles / c_s
        roof = dict(bound="hbm", kernel="pass_c", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9,
                    unit="GB/s", frac=achieved / PEAK_HBM,
                    traffic=measured_traffic("pass_c", head) if w.name == "disk1024_n1m" else None,
                    kernel_us=r["pass_c_us"], work_per_update=STATE_BYTES[head] // 2, work_unit="bytes")
    # HBM bytes the whole step moves (counters) against its algorithmic bytes
    st = measured_step_traffic(head) if w.name == "disk1024_n1m" else None
    r["step_traffic_bytes"] = st
    r["traffic_ratio"] = st / (STATE_BYTES[head] * w.n_particles) if st else None

    out = {
        "metric": "particle-updates/sec FP16 vs FP64 at <=0.5px track error; p99 frame latency",
        "value": r["updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "gpu_warmup_s": args.gpu_warmup_s,
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
        "kernel_source_sha256": kernel_source_hash(),
    }
    if variant:
        out["variant"] = variant
    if "f64" in res:
        out["speedup_f16_vs_f64"] = res["f64"]["seconds"] / res.get("f16", res["f64"])["seconds"]
    if "f32" in res and "f16" in res:
        out["speedup_f16_vs_f32"] = res["f32"]["seconds"] / res["f16"]["seconds"]
    def section(key, fn):
        # an optional section that fails is recorded, and the headline line
        # is still printed
        try:
            out[key] = fn()
            log(f"[bench] {key}: {json.dumps(out[key])}")
        except Exception as e:
            log(f"[bench] {key} failed: {e!r}")
            out[key] = {"error": repr(e)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    if not args.no_ablation:
        section("ablation", lambda: run_ablation(pf, torch, frames_dev, vid.centres, w,
                                                 min(args.steps, 40), args.warmup))
        section("resamplers", lambda: run_resamplers(pf, torch, frames_dev, vid.centres, w,
                                                     min(args.steps, 40), args.warmup))
        section("paper_sizes", lambda: run_paper_sizes(pf, torch, frames_dev, vid.centres, w,
                                                       min(args.steps, 40), args.warmup))
        section("resampler_bias", lambda: run_resampler_bias(pf, torch, pfsynth))
    if not args.no_ablation:
        def tune_headline():
            from paper_2308_00763_amd.tune import autotune
            r = autotune(w.n_particles, w.width, w.height, frames_dev, dtype=head, radius=w.radius,
                         x0=vid.centres[0][0], y0=vid.centres[0][1], drift=w.drift, sigma=w.sigma)
            r["default_threads"] = {"pass_a": 256, "pass_c": 256}
            return r
        section("autotune", tune_headline)
    if not args.no_track:
        section("accuracy", lambda: run_accuracy(pf, torch, pfsynth, modes))
    if args.large and args.large != "none":
        section("large", lambda: run_large(pf, torch, pfsynth, args, modes))
    if args.fleet:
        section("fleet", lambda: run_fleet(pf, torch, pfsynth, args.fleet, 256, 50, 40, 5))
    if args.serve_seconds > 0:
        hbm = tuple(float(x) for x in args.serve_hbm_gb.split(","))
        section("serving", lambda: run_serving(pf, torch, pfsynth, args.serve_seconds, 10.0, hbm_gb=hbm,
                                               admission=args.serve_admission))
        section("serving_closed_loop", lambda: run_serving_closed(pf, torch, pfsynth, 10.0, hbm_gb=hbm,
                                                                  admission=args.serve_admission))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        section("cpu_baseline", lambda: cpu_baseline(w, vid, args.cpu_budget, pfsynth))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
