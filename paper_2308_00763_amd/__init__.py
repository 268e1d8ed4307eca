"""Python binding of libpf: a reduced-precision SIR particle filter for object
tracking in greyscale video, with its per-frame step in HIP for AMD gfx950.

This module only marshals arguments to the C ABI declared in ``include/pf.h``
(same function names); every step of the filter runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace, frames) and streams.
If the library has not been built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")
# Workgroup sizes measured per (GPU architecture, dtype, particle-count
# bucket) by tune.py; installed in the library when it is loaded, read by
# filters created with PF_FLAG_TUNED.
TUNE_TABLE = os.path.join(_HERE, "tune_table.txt")

PF_OK = 0
PF_ERR_INVALID_ARG = 1
PF_ERR_WORKSPACE = 2
PF_ERR_HIP = 3
PF_ERR_STATE = 4

PF_F64, PF_F32, PF_F16, PF_BF16 = 0, 1, 2, 3
DTYPES = {"f64": PF_F64, "f32": PF_F32, "f16": PF_F16, "bf16": PF_BF16}
PF_LIK_MEAN, PF_LIK_SUM = 0, 1
PF_FLAG_DIAGNOSTICS = 1
PF_FLAG_NAIVE_LIKELIHOOD = 2
PF_FLAG_NAIVE_RESAMPLE = 4
PF_FLAG_NAIVE_HALF = 1 << 29
PF_THREADS_A_SHIFT = 8
PF_THREADS_C_SHIFT = 12
PF_FLAG_METROPOLIS = 1 << 16
PF_METROPOLIS_STEPS_SHIFT = 18
PF_FLAG_GUMBEL_MAX = 1 << 17
PF_FLAG_REJECTION = 1 << 28
PF_FLAG_STATE_ONLY = 1 << 26
PF_FLAG_TUNED = 1 << 30
PF_STATIC_SCRATCH_BYTES = 24 * 1024 * 1024 + 64 * 1024

PF_ABI_VERSION = 6

# Every function the C header declares (checked against include/pf.h by the tests).
EXPORTS = ("pf_workspace_bytes", "pf_member_bytes", "pf_init", "pf_step", "pf_step_static_scratch", "pf_estimate",
           "pf_estimate_async",
           "pf_export", "pf_export_step", "pf_import", "pf_destroy", "pf_last_error",
           "pf_abi_version", "pf_profile_start", "pf_profile_read",
           "pf_batch_workspace_bytes", "pf_batch_init", "pf_batch_step", "pf_batch_estimates",
           "pf_batch_estimates_async", "pf_batch_reinit", "pf_batch_filter", "pf_batch_destroy",
           "pf_tune_set", "pf_tune_load", "pf_tune_clear", "pf_tune_lookup", "pf_launch_config",
           "pf_batch_workspace_bytes_cap", "pf_batch_init_cap", "pf_batch_rebind")


class PfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpf error {code}: {msg}")
        self.code = code


class pf_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dtype", ctypes.c_int32),
        ("n_particles", ctypes.c_int64),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("disk_radius", ctypes.c_int32),
        ("fg", ctypes.c_int32),
        ("bg", ctypes.c_int32),
        ("lik_norm", ctypes.c_int32),
        ("kappa", ctypes.c_double),
        ("x0", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("drift_x", ctypes.c_double),
        ("drift_y", ctypes.c_double),
        ("sigma_x", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def lib():
    """The loaded libpf (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpf.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.pf_workspace_bytes.argtypes = [P(pf_params), P(ctypes.c_size_t)]
        L.pf_member_bytes.argtypes = [P(pf_params), P(ctypes.c_size_t)]
        L.pf_init.argtypes = [P(pf_params), vp, ctypes.c_size_t, vp, P(vp)]
        L.pf_step.argtypes = [vp, vp, ctypes.c_int64]
        L.pf_step_static_scratch.argtypes = [vp, vp, ctypes.c_int64]
        L.pf_estimate.argtypes = [vp, P(ctypes.c_double)]
        L.pf_estimate_async.argtypes = [vp, vp]
        L.pf_export.argtypes = [vp, vp, vp, vp, vp, P(ctypes.c_uint32)]
        L.pf_export_step.argtypes = [vp, vp, vp, vp]
        L.pf_import.argtypes = [vp, vp, vp, ctypes.c_uint32]
        L.pf_destroy.argtypes = [vp]
        L.pf_last_error.argtypes = []
        L.pf_last_error.restype = ctypes.c_char_p
        L.pf_abi_version.argtypes = []
        L.pf_profile_start.argtypes = [vp, ctypes.c_uint32]
        L.pf_profile_read.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_uint32)]
        L.pf_batch_workspace_bytes.argtypes = [P(pf_params), ctypes.c_int32, P(ctypes.c_size_t)]
        L.pf_batch_init.argtypes = [P(pf_params), ctypes.c_int32, vp, ctypes.c_size_t, vp, P(vp)]
        L.pf_batch_step.argtypes = [vp, vp, vp, vp]
        L.pf_batch_estimates.argtypes = [vp, vp]
        L.pf_batch_estimates_async.argtypes = [vp, vp]
        L.pf_batch_reinit.argtypes = [vp, ctypes.c_int32, P(pf_params)]
        L.pf_batch_filter.argtypes = [vp, ctypes.c_int32, P(vp)]
        L.pf_batch_destroy.argtypes = [vp]
        i32 = ctypes.c_int32
        L.pf_tune_set.argtypes = [ctypes.c_char_p, i32, i32, i32, i32]
        L.pf_tune_load.argtypes = [ctypes.c_char_p, P(i32)]
        L.pf_tune_clear.argtypes = []
        L.pf_tune_lookup.argtypes = [ctypes.c_char_p, i32, ctypes.c_int64, P(i32), P(i32)]
        L.pf_launch_config.argtypes = [vp, P(i32), P(i32)]
        L.pf_batch_workspace_bytes_cap.argtypes = [P(pf_params), i32, ctypes.c_int64, P(ctypes.c_size_t)]
        L.pf_batch_init_cap.argtypes = [P(pf_params), i32, ctypes.c_int64, vp, ctypes.c_size_t, vp, P(vp)]
        L.pf_batch_rebind.argtypes = [vp, i32, P(pf_params), vp, ctypes.c_size_t]
        for name in EXPORTS:
            if name != "pf_last_error":
                getattr(L, name).restype = ctypes.c_int
        if os.path.exists(TUNE_TABLE):
            n = i32()
            if L.pf_tune_load(TUNE_TABLE.encode(), ctypes.byref(n)) != PF_OK:
                raise PfError(PF_ERR_INVALID_ARG, L.pf_last_error().decode())
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PF_OK:
        raise PfError(rc, lib().pf_last_error().decode())


def threads_field(threads) -> int:
    """Field value of a threads-per-workgroup flag (None: 0, the default)."""
    if threads is None:
        return 0
    v = int(threads).bit_length() - 6
    if threads <= 0 or threads != 1 << (v + 5) or not 1 <= v <= 5:
        raise ValueError(f"threads per workgroup must be a power of two in [64, 1024], got {threads}")
    return v


def make_params(n, width, height, dtype="f64", radius=5, x0=0.0, y0=0.0, drift=(1.0, -2.0),
                sigma=(5.0, 2.0), seed=0, stream_id=0, fg=228, bg=100, kappa=50.0,
                lik_norm=PF_LIK_MEAN, diagnostics=False, naive_likelihood=False,
                naive_resample=False, threads_a=None, threads_c=None,
                metropolis_steps=0, gumbel_max=False, rejection_trials=0,
                state_only=False, naive_half=False, tuned=False) -> pf_params:
    """Parameters of one filter.  rejection_trials > 0 selects rejection
    resampling with at most that many trials per slot (a multiple of 64 up
    to 16320).  tuned=True takes the workgroup sizes from the library's
    tuning table (threads_a and threads_c must then be None)."""
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    if not 0 <= int(metropolis_steps) <= 255:
        raise ValueError(f"metropolis_steps must be in [0, 255], got {metropolis_steps}")
    rj = int(rejection_trials)
    if rj and (rj % 64 or not 64 <= rj <= 64 * 255):
        raise ValueError(f"rejection_trials must be a multiple of 64 in [64, 16320], got {rejection_trials}")
    flags = ((PF_FLAG_DIAGNOSTICS if diagnostics else 0)
             | (PF_FLAG_NAIVE_LIKELIHOOD if naive_likelihood else 0)
             | (PF_FLAG_NAIVE_RESAMPLE if naive_resample else 0)
             | (threads_field(threads_a) << PF_THREADS_A_SHIFT)
             | (threads_field(threads_c) << PF_THREADS_C_SHIFT)
             | ((PF_FLAG_METROPOLIS | (int(metropolis_steps) << PF_METROPOLIS_STEPS_SHIFT))
                if metropolis_steps else 0)
             | (PF_FLAG_GUMBEL_MAX if gumbel_max else 0)
             | ((PF_FLAG_REJECTION | ((rj // 64) << PF_METROPOLIS_STEPS_SHIFT)) if rj else 0)
             | (PF_FLAG_STATE_ONLY if state_only else 0)
             | (PF_FLAG_NAIVE_HALF if naive_half else 0)
             | (PF_FLAG_TUNED if tuned else 0))
    return pf_params(ctypes.sizeof(pf_params), dt, int(n), int(width), int(height), int(radius),
                     int(fg), int(bg), int(lik_norm), float(kappa), float(x0), float(y0),
                     float(drift[0]), float(drift[1]), float(sigma[0]), float(sigma[1]),
                     int(seed) & (2**64 - 1), int(stream_id), flags)


# ---------------------------------------------------------------------------
# C-ABI functions under their C names (argument marshalling only).

def pf_workspace_bytes(p: pf_params) -> int:
    out = ctypes.c_size_t()
    _check(lib().pf_workspace_bytes(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def pf_member_bytes(p: pf_params) -> int:
    out = ctypes.c_size_t()
    _check(lib().pf_member_bytes(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def pf_init(p: pf_params, d_workspace: int, workspace_bytes: int, hip_stream: int):
    h = ctypes.c_void_p()
    _check(lib().pf_init(ctypes.byref(p), ctypes.c_void_p(d_workspace), workspace_bytes,
                         ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h


def pf_step(h, d_frame: int, row_pitch: int):
    _check(lib().pf_step(h, ctypes.c_void_p(d_frame), int(row_pitch)))


def pf_step_static_scratch(h, d_frame: int, row_pitch: int):
    _check(lib().pf_step_static_scratch(h, ctypes.c_void_p(d_frame), int(row_pitch)))


def pf_estimate(h):
    out = (ctypes.c_double * 2)()
    _check(lib().pf_estimate(h, out))
    return float(out[0]), float(out[1])


def pf_estimate_async(h, d_out: int):
    _check(lib().pf_estimate_async(h, ctypes.c_void_p(d_out)))


def _np_ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def pf_export(h, n: int, diagnostics: bool = False):
    x = np.zeros(n)
    y = np.zeros(n)
    w = np.zeros(n) if diagnostics else None
    anc = np.zeros(n, dtype=np.int32) if diagnostics else None
    t = ctypes.c_uint32()
    _check(lib().pf_export(h, _np_ptr(x), _np_ptr(y), _np_ptr(w), _np_ptr(anc), ctypes.byref(t)))
    return dict(x=x, y=y, w=w, anc=anc, t=t.value)


def pf_export_step(h, n: int, diagnostics: bool = False):
    x = np.zeros(n)
    y = np.zeros(n)
    s = np.zeros(n, dtype=np.int32) if diagnostics else None
    _check(lib().pf_export_step(h, _np_ptr(x), _np_ptr(y), _np_ptr(s)))
    return dict(x_prop=x, y_prop=y, disk_sum=s)


def pf_import(h, x, y, t: int):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    _check(lib().pf_import(h, _np_ptr(x), _np_ptr(y), int(t)))


def pf_destroy(h):
    _check(lib().pf_destroy(h))


def pf_last_error() -> str:
    return lib().pf_last_error().decode()


def pf_abi_version() -> int:
    return lib().pf_abi_version()


def pf_profile_start(h, max_steps: int):
    _check(lib().pf_profile_start(h, int(max_steps)))


def pf_profile_read(h):
    """(pass A ms, combine ms, pass C ms, steps) summed over the recorded steps."""
    out = (ctypes.c_double * 3)()
    steps = ctypes.c_uint32()
    _check(lib().pf_profile_read(h, out, ctypes.byref(steps)))
    return float(out[0]), float(out[1]), float(out[2]), steps.value


def _params_array(params):
    arr = (pf_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def pf_batch_workspace_bytes(params) -> int:
    arr = _params_array(params)
    out = ctypes.c_size_t()
    _check(lib().pf_batch_workspace_bytes(arr, len(params), ctypes.byref(out)))
    return out.value


def pf_batch_init(params, d_workspace: int, workspace_bytes: int, hip_stream: int):
    arr = _params_array(params)
    b = ctypes.c_void_p()
    _check(lib().pf_batch_init(arr, len(params), ctypes.c_void_p(d_workspace), workspace_bytes,
                               ctypes.c_void_p(hip_stream), ctypes.byref(b)))
    return b


def pf_batch_workspace_bytes_cap(params, max_tiles: int) -> int:
    arr = _params_array(params)
    out = ctypes.c_size_t()
    _check(lib().pf_batch_workspace_bytes_cap(arr, len(params), int(max_tiles), ctypes.byref(out)))
    return out.value


def pf_batch_init_cap(params, max_tiles: int, d_workspace: int, workspace_bytes: int, hip_stream: int):
    arr = _params_array(params)
    b = ctypes.c_void_p()
    _check(lib().pf_batch_init_cap(arr, len(params), int(max_tiles), ctypes.c_void_p(d_workspace),
                                   workspace_bytes, ctypes.c_void_p(hip_stream), ctypes.byref(b)))
    return b


def pf_batch_rebind(b, k: int, p: pf_params, d_share: int, share_bytes: int):
    _check(lib().pf_batch_rebind(b, int(k), ctypes.byref(p), ctypes.c_void_p(d_share), int(share_bytes)))


def pf_batch_step(b, d_frames, pitches, active=None):
    """d_frames: uint64 array of device pointers; pitches: int64 array;
    active: uint8 array or None (all)."""
    fr = np.ascontiguousarray(d_frames, dtype=np.uint64)
    pi = np.ascontiguousarray(pitches, dtype=np.int64)
    ac = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    _check(lib().pf_batch_step(b, _np_ptr(fr), _np_ptr(pi), _np_ptr(ac)))


def pf_batch_estimates(b, n: int):
    out = np.zeros(2 * n)
    _check(lib().pf_batch_estimates(b, _np_ptr(out)))
    return out.reshape(n, 2)


def pf_batch_estimates_async(b, d_out: int):
    _check(lib().pf_batch_estimates_async(b, ctypes.c_void_p(d_out)))


def pf_batch_reinit(b, k: int, p: pf_params):
    _check(lib().pf_batch_reinit(b, int(k), ctypes.byref(p)))


def pf_batch_filter(b, k: int):
    h = ctypes.c_void_p()
    _check(lib().pf_batch_filter(b, int(k), ctypes.byref(h)))
    return h


def pf_batch_destroy(b):
    _check(lib().pf_batch_destroy(b))


# ---------------------------------------------------------------------------
# Convenience wrapper: workspace and stream from PyTorch.

def pf_tune_set(arch: str, dtype, bucket: int, threads_a: int, threads_c: int):
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _check(lib().pf_tune_set(arch.encode(), dt, int(bucket), int(threads_a), int(threads_c)))


def pf_tune_load(path: str) -> int:
    n = ctypes.c_int32()
    _check(lib().pf_tune_load(path.encode(), ctypes.byref(n)))
    return n.value


def pf_tune_clear():
    _check(lib().pf_tune_clear())


def pf_tune_lookup(arch: str, dtype, n: int):
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    ta, tc = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().pf_tune_lookup(arch.encode(), dt, int(n), ctypes.byref(ta), ctypes.byref(tc)))
    return ta.value, tc.value


def pf_launch_config(h):
    ta, tc = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().pf_launch_config(h, ctypes.byref(ta), ctypes.byref(tc)))
    return ta.value, tc.value


class Filter:
    """One particle filter with a torch-allocated workspace on `device`."""

    def __init__(self, params: pf_params, device="cuda:0", stream=None):
        import torch
        self.params = params
        self.n = params.n_particles
        self.diagnostics = bool(params.flags & PF_FLAG_DIAGNOSTICS)
        self.device = torch.device(device)
        nbytes = pf_workspace_bytes(params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = pf_init(params, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def step(self, frame):
        """frame: (H, W) uint8 CUDA tensor (row pitch from its stride)."""
        assert frame.dtype.itemsize == 1 and frame.dim() == 2 and frame.stride(1) == 1
        assert frame.is_cuda
        if self.params.flags & PF_FLAG_STATE_ONLY:
            pf_step_static_scratch(self.handle, frame.data_ptr(), frame.stride(0))
        else:
            pf_step(self.handle, frame.data_ptr(), frame.stride(0))

    def estimate(self):
        return pf_estimate(self.handle)

    def launch_config(self):
        """(pass A threads, pass C threads) the filter launches with."""
        return pf_launch_config(self.handle)

    def export(self):
        return pf_export(self.handle, self.n, self.diagnostics)

    def export_step(self):
        return pf_export_step(self.handle, self.n, self.diagnostics)

    def load(self, x, y, t):
        pf_import(self.handle, x, y, t)

    def close(self):
        if self.handle is not None:
            pf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of filters in one torch-allocated workspace on `device`."""

    def __init__(self, params, device="cuda:0", stream=None, max_tiles=0):
        """max_tiles: tile capacity of the batch's plan (0: the members' own
        tiles), room for members rebound to larger filters."""
        import torch
        self.params = list(params)
        self.n = len(self.params)
        self.device = torch.device(device)
        nbytes = pf_batch_workspace_bytes_cap(self.params, max_tiles)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = pf_batch_init_cap(self.params, max_tiles, self.workspace.data_ptr(), nbytes,
                                        self.stream.cuda_stream)

    def step(self, frames, active=None):
        """frames: list of n (H_k, W_k) uint8 CUDA tensors (None where inactive)."""
        ptrs = np.zeros(self.n, dtype=np.uint64)
        pitches = np.zeros(self.n, dtype=np.int64)
        for k, f in enumerate(frames):
            if f is None:
                continue
            assert f.dtype.itemsize == 1 and f.dim() == 2 and f.stride(1) == 1 and f.is_cuda
            ptrs[k] = f.data_ptr()
            pitches[k] = f.stride(0)
        pf_batch_step(self.handle, ptrs, pitches, active)

    def step_ptrs(self, ptrs, pitches, active=None):
        pf_batch_step(self.handle, ptrs, pitches, active)

    def estimates(self):
        return pf_batch_estimates(self.handle, self.n)

    def filter(self, k: int):
        return pf_batch_filter(self.handle, k)

    def reinit(self, k: int, params: pf_params):
        pf_batch_reinit(self.handle, k, params)
        self.params[k] = params

    def rebind(self, k: int, params: pf_params, d_share: int, share_bytes: int):
        """Filter k re-initialised on a workspace share the caller owns."""
        pf_batch_rebind(self.handle, k, params, d_share, share_bytes)
        self.params[k] = params

    def export(self, k: int):
        p = self.params[k]
        return pf_export(self.filter(k), p.n_particles, bool(p.flags & PF_FLAG_DIAGNOSTICS))

    def close(self):
        if self.handle is not None:
            pf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
