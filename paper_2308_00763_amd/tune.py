"""Workgroup-size autotuner for the single-filter step.

Pass A (1024 particles per workgroup, 128/256/512 threads) and pass C (one
tile per workgroup, 64-1024 threads) are timed with the library's own
per-kernel events on the caller's frames, and the fastest pair is returned
as flags for pf_params.  Results do not depend on pass C's size; pass A's size
changes only the rounding order of the tile-local prefix sums, so a tuned
filter keeps the parity of the default one.  Choices are made per
(precision, particle-count bucket), never per batch composition: batches run
the default step.
"""
from __future__ import annotations

import math

from . import (PF_THREADS_A_SHIFT, PF_THREADS_C_SHIFT, Filter, lib, make_params, pf_profile_read,
               pf_profile_start, threads_field)

PASS_A_THREADS = (128, 256, 512)
PASS_C_THREADS = (128, 256, 512, 1024)


def bucket(n: int) -> int:
    """Particle-count bucket: ceil(log2 N)."""
    return max(0, math.ceil(math.log2(max(1, n))))


def _time(params, frames, steps, warmup):
    """Mean microseconds per step of pass A and pass C (dispatch-stamped
    events) over `steps` steps after `warmup`, stepping through `frames`."""
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
    a_ms, _, c_ms, n = pf_profile_read(f.handle)
    f.close()
    return 1e3 * a_ms / n, 1e3 * c_ms / n


def autotune(n, width, height, frames, dtype="f16", radius=5, steps=20, warmup=5, **model):
    """Time every pass-A and pass-C size on `frames` ((T, H, W) uint8 device
    tensor, T >= 2) for a filter of n particles; returns
    dict(threads_a, threads_c, flags, pass_a_us, pass_c_us, table)."""
    table = {"pass_a": {}, "pass_c": {}}
    for ta in PASS_A_THREADS:
        p = make_params(n, width, height, dtype, radius=radius, threads_a=ta, **model)
        table["pass_a"][ta] = _time(p, frames, steps, warmup)[0]
    for tc in PASS_C_THREADS:
        p = make_params(n, width, height, dtype, radius=radius, threads_c=tc, **model)
        table["pass_c"][tc] = _time(p, frames, steps, warmup)[1]
    ta = min(table["pass_a"], key=table["pass_a"].get)
    tc = min(table["pass_c"], key=table["pass_c"].get)
    flags = (threads_field(ta) << PF_THREADS_A_SHIFT) | (threads_field(tc) << PF_THREADS_C_SHIFT)
    return dict(threads_a=ta, threads_c=tc, flags=flags, pass_a_us=table["pass_a"][ta],
                pass_c_us=table["pass_c"][tc], bucket=bucket(n), dtype=dtype, table=table)
