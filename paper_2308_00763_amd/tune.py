"""Workgroup-size autotuner for the single-filter step, and the tuning table
it writes.

Pass A (1024 particles per workgroup, 128/256/512 threads) and pass C (one
tile per workgroup at a time, 64-1024 threads) sizes are each timed as whole
steps with the library's own per-kernel events (at the default sizes an FP32
or FP64 filter of at most 2^20 particles resamples inside the next pass A
instead of in pass C, so a size is worth what it does to the step), and the
fastest sizes are kept.
Results do not depend on pass C's size; pass A's size changes only the
rounding order of the tile-local prefix sums.  This is the threads-per-block study of the paper
(Sec. 5) turned into configuration: ``sweep`` measures every (dtype,
particle-count bucket) on the GPU it runs on and ``write_table`` stores the
result as the text table that the library reads (``pf_tune_load``) and
consults for filters created with ``PF_FLAG_TUNED`` -- alone or in a batch,
where each member runs pass A at its own tuned size.

Command that writes the shipped table (on the GPU it is meant for):

    python -m paper_2308_00763_amd.tune --write paper_2308_00763_amd/tune_table.txt
"""
from __future__ import annotations

import argparse
import math
import statistics
import sys

from . import (PF_THREADS_A_SHIFT, PF_THREADS_C_SHIFT, Filter, lib, make_params, pf_profile_read,
               pf_profile_start, threads_field)

PASS_A_THREADS = (128, 256, 512)
PASS_C_THREADS = (128, 256, 512, 1024)
DEFAULT_A, DEFAULT_C = 256, 256

# buckets ceil(log2 N) of the shipped table (2^10 ... 2^24 particles)
TABLE_BUCKETS = (10, 12, 14, 16, 18, 20, 22, 24)
TABLE_DTYPES = ("f16", "bf16", "f32", "f64")
# a size other than the default is kept only when it is at least this much
# faster than the default (run-to-run spread of the timings is about 1-2 %)
MIN_GAIN = 0.03


def bucket(n: int) -> int:
    """Particle-count bucket: ceil(log2 N)."""
    return max(0, math.ceil(math.log2(max(1, n))))


def _time(params, frames, steps, warmup):
    """Mean microseconds per step of pass A and of the rest of the step (the
    combine and pass C; no pass C for a filter that defers its resampling),
    from dispatch-stamped events over `steps` steps after `warmup`, stepping
    through `frames`."""
    import ctypes
    f = Filter(params)
    L = lib()
    T = frames.shape[0]
    ptr = [ctypes.c_void_p(frames[t % (T - 1) + 1].data_ptr()) for t in range(warmup + steps)]
    pitch = int(frames.stride(1))
    for t in range(warmup):
        L.pf_step(f.handle, ptr[t], pitch)
    pf_profile_start(f.handle, steps)
    for t in range(warmup, warmup + steps):
        L.pf_step(f.handle, ptr[t], pitch)
    a_ms, m_ms, c_ms, n = pf_profile_read(f.handle)
    f.close()
    return 1e3 * a_ms / n, 1e3 * (m_ms + c_ms) / n


def autotune(n, width, height, frames, dtype="f16", radius=5, steps=20, warmup=5, rounds=1, **model):
    """Time every pass-A and pass-C size on `frames` ((T, H, W) uint8 device
    tensor, T >= 2) for a filter of n particles, `rounds` interleaved rounds
    (median per size); returns dict(threads_a, threads_c, flags, pass_a_us,
    pass_c_us, table): table["pass_a"] / table["pass_c"] hold the step's
    kernel time (us) per pass-A / pass-C size, the other size left at its
    default (given as no size, so that a filter that defers its resampling
    at the default sizes is timed that way), and pass_a_us / pass_c_us the
    fastest of each."""
    times_a = {ta: [] for ta in PASS_A_THREADS}
    times_c = {tc: [] for tc in PASS_C_THREADS}
    for _ in range(rounds):
        for ta in PASS_A_THREADS:
            p = make_params(n, width, height, dtype, radius=radius, threads_a=None if ta == DEFAULT_A else ta,
                            **model)
            times_a[ta].append(sum(_time(p, frames, steps, warmup)))
        for tc in PASS_C_THREADS:
            p = make_params(n, width, height, dtype, radius=radius, threads_c=None if tc == DEFAULT_C else tc,
                            **model)
            times_c[tc].append(sum(_time(p, frames, steps, warmup)))
    table = {"pass_a": {k: statistics.median(v) for k, v in times_a.items()},
             "pass_c": {k: statistics.median(v) for k, v in times_c.items()}}
    ta = min(table["pass_a"], key=table["pass_a"].get)
    tc = min(table["pass_c"], key=table["pass_c"].get)
    flags = (threads_field(ta) << PF_THREADS_A_SHIFT) | (threads_field(tc) << PF_THREADS_C_SHIFT)
    return dict(threads_a=ta, threads_c=tc, flags=flags, pass_a_us=table["pass_a"][ta],
                pass_c_us=table["pass_c"][tc], bucket=bucket(n), dtype=dtype, table=table)


def choose(res: dict) -> tuple[int, int]:
    """Table sizes from an autotune result: the fastest size when it beats the
    default by at least MIN_GAIN, else 0 (the default)."""
    out = []
    for key, best, dflt in (("pass_a", res["threads_a"], DEFAULT_A), ("pass_c", res["threads_c"], DEFAULT_C)):
        t = res["table"][key]
        out.append(best if best != dflt and t[best] <= (1.0 - MIN_GAIN) * t[dflt] else 0)
    return out[0], out[1]


def sweep(frames, width, height, dtypes=TABLE_DTYPES, buckets=TABLE_BUCKETS, radius=5, steps=20, warmup=5,
          rounds=3, log=None, **model):
    """autotune at N = 2^b for every dtype and bucket b; returns a list of
    dict(dtype, bucket, threads_a, threads_c, result)."""
    rows = []
    for dt in dtypes:
        for b in buckets:
            res = autotune(1 << b, width, height, frames, dtype=dt, radius=radius, steps=steps,
                           warmup=warmup, rounds=rounds, **model)
            ta, tc = choose(res)
            rows.append(dict(dtype=dt, bucket=b, threads_a=ta, threads_c=tc, result=res))
            if log:
                log(f"[tune] {dt} 2^{b}: pass A {res['table']['pass_a']} pass C {res['table']['pass_c']} "
                    f"-> ({ta}, {tc})")
    return rows


def write_table(path, arch, rows, header=""):
    """Write the rows of `sweep` as a table file for pf_tune_load."""
    with open(path, "w") as f:
        for line in header.splitlines():
            f.write(f"# {line}\n")
        f.write("# arch dtype bucket threads_a threads_c   (0: default size; in the comment, us per step by "
                "pass-A size | by pass-C size)\n")
        for r in rows:
            t = r["result"]["table"]
            pa = " ".join(f"{k}:{v:.2f}" for k, v in t["pass_a"].items())
            pc = " ".join(f"{k}:{v:.2f}" for k, v in t["pass_c"].items())
            f.write(f"{arch} {r['dtype']} {r['bucket']} {r['threads_a']} {r['threads_c']}"
                    f"   # A {pa} | C {pc}\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--write", required=True, metavar="PATH", help="table file to write")
    ap.add_argument("--dtypes", default=",".join(TABLE_DTYPES))
    ap.add_argument("--buckets", default=",".join(map(str, TABLE_BUCKETS)))
    ap.add_argument("--rounds", type=int, default=3)
    args = ap.parse_args(argv)
    import torch

    import pfsynth  # the seeded synthetic videos (repository root)
    w = pfsynth.WORKLOADS["disk1024_n1m"]
    vid = pfsynth.workload_video(w, frames=32)
    frames = torch.from_numpy(vid.frames).to("cuda:0")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    rows = sweep(frames, w.width, w.height, dtypes=args.dtypes.split(","),
                 buckets=[int(b) for b in args.buckets.split(",")], radius=w.radius, rounds=args.rounds,
                 log=log, x0=vid.centres[0][0], y0=vid.centres[0][1], drift=w.drift, sigma=w.sigma,
                 seed=w.filter_seed)
    header = (f"Workgroup sizes for {arch}, measured by paper_2308_00763_amd.tune on the {w.width}x{w.height} "
              f"moving-disk video (r = {w.radius}),\nN = 2^bucket, median of {args.rounds} interleaved rounds "
              f"of 20 timed steps per size; a size other than the default\nis kept only when at least "
              f"{int(MIN_GAIN * 100)} % faster than the default.")
    write_table(args.write, arch, rows, header)
    print(f"wrote {len(rows)} entries to {args.write}", flush=True)


if __name__ == "__main__":
    main()
