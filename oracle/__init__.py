"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle (pf_oracle.c).

The oracle is the plain, sequential, double-precision SIR step of the
half-precision particle filter paper (arXiv:2308.00763, Sec. 4, Eq. (1)-(5) and
the normalizing / systematic-resampling paragraphs).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may use
it; the product library never loads it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_SRC_OMP = os.path.join(_HERE, "pf_oracle_omp.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_BUILD, "liboracle_omp.so")

MEAN = 0
SUM = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, glibc libm): the
    sequential build used for parity, and the OpenMP build used only to time
    the oracle on every host core."""
    os.makedirs(_BUILD, exist_ok=True)
    for src, path, extra in ((_SRC, _LIB_PATH, []), (_SRC_OMP, _LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math"] + extra +
                ["-fPIC", "-shared", src, "-lm", "-o", tmp])
            os.replace(tmp, path)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("radius", ctypes.c_int32),
        ("fg", ctypes.c_int32),
        ("bg", ctypes.c_int32),
        ("lik_norm", ctypes.c_int32),
        ("kappa", ctypes.c_double),
        ("drift_x", ctypes.c_double),
        ("drift_y", ctypes.c_double),
        ("sigma_x", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(Params)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.or_philox_words.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [u32p]
        L.or_uniform53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.or_uniform53.restype = ctypes.c_double
        L.or_normal_pair.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, dp, dp]
        L.or_u0.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.or_u0.restype = ctypes.c_double
        L.or_disk.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.or_disk.restype = ctypes.c_int
        L.or_propagate.argtypes = [pp, ctypes.c_uint32, dp, dp]
        L.or_likelihood_one.argtypes = [pp, u8p, ctypes.c_int64, ctypes.c_double, ctypes.c_double]
        L.or_likelihood_one.restype = ctypes.c_double
        L.or_likelihood.argtypes = [pp, u8p, ctypes.c_int64, dp, dp, dp]
        L.or_reweight_resample.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double,
                                           dp, dp, ip, dp, dp, dp]
        L.or_step.argtypes = [pp, ctypes.c_uint32, u8p, ctypes.c_int64, dp, dp, dp, dp, dp,
                              dp, ip, dp]
        L.or_run.argtypes = [pp, u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                             ctypes.c_double, dp, dp, dp]
        L.or_metropolis.argtypes = [ctypes.c_int64, dp, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_uint32, ctypes.c_uint32, ip, dp]
        L.or_gumbel_max.argtypes = [ctypes.c_int64, dp, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, ip, dp]
        L.or_rejection.argtypes = [ctypes.c_int64, dp, ctypes.c_int32, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_uint32, ip, dp, ip]
        _lib = L
    return _lib


_lib_omp = None


def lib_omp():
    """The OpenMP timing build (pf_oracle_omp.c)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_OMP_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_step_omp.argtypes = [ctypes.POINTER(Params), ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64,
                                  dp, dp, dp, dp, dp, dp, dp]
        L.or_step_omp.restype = ctypes.c_int
        L.or_omp_set_threads.argtypes = [ctypes.c_int]
        L.or_omp_max_threads.restype = ctypes.c_int
        _lib_omp = L
    return _lib_omp


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_params(n, width, height, radius=5, fg=228, bg=100, lik_norm=MEAN, kappa=50.0,
                drift=(1.0, -2.0), sigma=(5.0, 2.0), seed=0, stream_id=0) -> Params:
    return Params(int(n), int(width), int(height), int(radius), int(fg), int(bg),
                  int(lik_norm), float(kappa), float(drift[0]), float(drift[1]),
                  float(sigma[0]), float(sigma[1]), int(seed), int(stream_id))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                           _ptr(out, ctypes.c_uint32))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64),
                           _ptr(out, ctypes.c_uint64))
    return out


def philox_words(seed, c0, c1, c2, c3) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox_words(seed, c0, c1, c2, c3, _ptr(out, ctypes.c_uint32))
    return out


def uniform53(hi, lo) -> float:
    return lib().or_uniform53(hi, lo)


def normal_pair(seed, k, t, stream_id):
    zx = ctypes.c_double()
    zy = ctypes.c_double()
    lib().or_normal_pair(seed, k, t, stream_id, ctypes.byref(zx), ctypes.byref(zy))
    return zx.value, zy.value


def u0(seed, stream_id, t) -> float:
    return lib().or_u0(seed, stream_id, t)


def disk(r):
    n = lib().or_disk(r, None, None, 0)
    dx = (ctypes.c_int * n)()
    dy = (ctypes.c_int * n)()
    lib().or_disk(r, dx, dy, n)
    return np.array(list(dx), dtype=np.int64), np.array(list(dy), dtype=np.int64)


def propagate(p: Params, t, x, y):
    x = np.array(x, dtype=np.float64)
    y = np.array(y, dtype=np.float64)
    assert x.size == p.n and y.size == p.n
    lib().or_propagate(ctypes.byref(p), t, _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double))
    return x, y


def likelihood(p: Params, frame, x, y) -> np.ndarray:
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    assert frame.shape == (p.height, p.width)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    L = np.zeros(x.size, dtype=np.float64)
    q = make_params(x.size, p.width, p.height, p.radius, p.fg, p.bg, p.lik_norm, p.kappa,
                    (p.drift_x, p.drift_y), (p.sigma_x, p.sigma_y), p.seed, p.stream_id)
    lib().or_likelihood(ctypes.byref(q), _ptr(frame, ctypes.c_uint8), frame.shape[1],
                        _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                        _ptr(L, ctypes.c_double))
    return L


def reweight_resample(L, x, y, u0_value, w_prev=None):
    """O6-O12 given log-likelihoods.  Returns dict(w, cdf, anc, x, y, est)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = L.size
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if w_prev is None:
        w_prev = np.full(n, 1.0 / n)
    w_prev = np.ascontiguousarray(w_prev, dtype=np.float64)
    w = np.zeros(n)
    cdf = np.zeros(n)
    anc = np.zeros(n, dtype=np.int32)
    xo = np.zeros(n)
    yo = np.zeros(n)
    est = np.zeros(2)
    lib().or_reweight_resample(n, _ptr(L, ctypes.c_double), _ptr(w_prev, ctypes.c_double),
                               _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                               float(u0_value), _ptr(w, ctypes.c_double),
                               _ptr(cdf, ctypes.c_double), _ptr(anc, ctypes.c_int32),
                               _ptr(xo, ctypes.c_double), _ptr(yo, ctypes.c_double),
                               _ptr(est, ctypes.c_double))
    return dict(w=w, cdf=cdf, anc=anc, x=xo, y=yo, est=est)


def step(p: Params, t, frame, x, y):
    """One SIR step.  Returns dict(x, y, x_prop, y_prop, L, w, anc, est)."""
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    assert frame.shape == (p.height, p.width)
    n = p.n
    x = np.array(x, dtype=np.float64)
    y = np.array(y, dtype=np.float64)
    assert x.size == n and y.size == n
    xp = np.zeros(n)
    yp = np.zeros(n)
    L = np.zeros(n)
    w = np.zeros(n)
    anc = np.zeros(n, dtype=np.int32)
    est = np.zeros(2)
    lib().or_step(ctypes.byref(p), t, _ptr(frame, ctypes.c_uint8), frame.shape[1],
                  _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                  _ptr(xp, ctypes.c_double), _ptr(yp, ctypes.c_double),
                  _ptr(L, ctypes.c_double), _ptr(w, ctypes.c_double),
                  _ptr(anc, ctypes.c_int32), _ptr(est, ctypes.c_double))
    return dict(x=x, y=y, x_prop=xp, y_prop=yp, L=L, w=w, anc=anc, est=est)


class OmpStepper:
    """Steps of one filter with the OpenMP timing build, reusing its work
    arrays; x, y hold the particles after the latest step.  `threads` > 0
    sets OpenMP's thread count for the process."""

    def __init__(self, p: Params, x, y, threads: int = 0):
        self.p = p
        self.x = np.array(x, dtype=np.float64)
        self.y = np.array(y, dtype=np.float64)
        assert self.x.size == p.n and self.y.size == p.n
        self.xp = np.zeros(p.n)
        self.yp = np.zeros(p.n)
        self.L = np.zeros(p.n)
        self.P = np.zeros(p.n)
        self.est = np.zeros(2)
        if threads > 0:
            lib_omp().or_omp_set_threads(int(threads))
        self.threads = 0

    def step(self, t, frame):
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        assert frame.shape == (self.p.height, self.p.width)
        d = ctypes.c_double
        self.threads = lib_omp().or_step_omp(
            ctypes.byref(self.p), t, _ptr(frame, ctypes.c_uint8), frame.shape[1],
            _ptr(self.x, d), _ptr(self.y, d), _ptr(self.xp, d), _ptr(self.yp, d),
            _ptr(self.L, d), _ptr(self.P, d), _ptr(self.est, d))
        return self.est.copy()


def run(p: Params, video, x0, y0):
    """Run over frames 1..T-1.  Returns (estimates (T, 2), final x, final y)."""
    video = np.ascontiguousarray(video, dtype=np.uint8)
    T, H, W = video.shape
    assert (H, W) == (p.height, p.width)
    x = np.zeros(p.n)
    y = np.zeros(p.n)
    est = np.zeros(2 * T)
    lib().or_run(ctypes.byref(p), _ptr(video, ctypes.c_uint8), W, T, float(x0), float(y0),
                 _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double), _ptr(est, ctypes.c_double))
    return est.reshape(T, 2), x, y


def metropolis(L, B: int, seed: int, stream_id: int, t: int):
    """Metropolis resampling of log-likelihoods L with B steps per slot
    (pf_oracle.c, or_metropolis).  Returns (ancestors, margins)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = L.size
    anc = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n)
    lib().or_metropolis(n, _ptr(L, ctypes.c_double), int(B), int(seed), int(stream_id), int(t),
                        _ptr(anc, ctypes.c_int32), _ptr(margin, ctypes.c_double))
    return anc, margin


def gumbel_max(L, seed: int, stream_id: int, t: int):
    """Gumbel-max multinomial resampling of log-likelihoods L (pf_oracle.c,
    or_gumbel_max).  Returns (ancestors, margins)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = L.size
    anc = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n)
    lib().or_gumbel_max(n, _ptr(L, ctypes.c_double), int(seed), int(stream_id), int(t),
                        _ptr(anc, ctypes.c_int32), _ptr(margin, ctypes.c_double))
    return anc, margin


def rejection(L, cap: int, seed: int, stream_id: int, t: int):
    """Rejection resampling of log-likelihoods L with at most `cap` trials per
    slot (pf_oracle.c, or_rejection).  Returns (ancestors, margins, trials)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = L.size
    anc = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n)
    trials = np.zeros(n, dtype=np.int32)
    lib().or_rejection(n, _ptr(L, ctypes.c_double), int(cap), int(seed), int(stream_id), int(t),
                       _ptr(anc, ctypes.c_int32), _ptr(margin, ctypes.c_double),
                       _ptr(trials, ctypes.c_int32))
    return anc, margin, trials
