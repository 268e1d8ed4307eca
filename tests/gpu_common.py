"""Shared helpers of the GPU parity tests: teacher-forced stepping of the HIP
filter against the FP64 CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2308_00763_amd as pf

PIX_TIE = 1e-9   # a coordinate this close to a half-integer may round either way
CDF_TIE = 1e-12  # a stratum point this close to a CDF value may fall either side


def oracle_params(n, W, H, r, drift=(1.0, -2.0), sigma=(5.0, 2.0), seed=0, stream_id=0,
                  lik_norm=0):
    return oracle.make_params(n, W, H, radius=r, drift=drift, sigma=sigma, seed=seed,
                              stream_id=stream_id, lik_norm=lik_norm)


def oracle_step_parts(op, t, frame, x, y):
    """The oracle's step, keeping every intermediate the comparison needs."""
    xp, yp = oracle.propagate(op, t, x, y)
    L = oracle.likelihood(op, frame, xp, yp)
    u0 = oracle.u0(op.seed, op.stream_id, t)
    ref = oracle.reweight_resample(L, xp, yp, u0)
    nd = oracle.disk(op.radius)[0].size
    denom = op.kappa * nd if op.lik_norm == 0 else op.kappa
    ref.update(x_prop=xp, y_prop=yp, L=L, u0=u0, S=np.rint(L * denom).astype(np.int64))
    return ref


def near_half(v, tol=PIX_TIE):
    return np.abs((v - 0.5) - np.round(v - 0.5)) < tol


def anc_ties(ref, n):
    """Slots whose stratum point lies within CDF_TIE of a CDF value next to
    the oracle's ancestor (either side may be chosen)."""
    j = np.arange(n)
    u = (j + ref["u0"]) / n
    C = ref["cdf"]
    a = ref["anc"]
    lo = np.where(a > 0, C[np.maximum(a - 1, 0)], -1.0)
    return (np.abs(u - C[a]) <= CDF_TIE) | (np.abs(u - lo) <= CDF_TIE)


def compare_f64_step(got, gs, est, ref, n, check_anc=True):
    """Element-wise parity of one teacher-forced FP64 step; returns counts of
    the mismatches that the tie rules excuse."""
    # propagation: same random stream, libm-level differences only
    assert np.max(np.abs(gs["x_prop"] - ref["x_prop"])) <= 1e-9
    assert np.max(np.abs(gs["y_prop"] - ref["y_prop"])) <= 1e-9
    # disk sums: integers, exact unless the pixel rounding is a tie
    bad = gs["disk_sum"].astype(np.int64) != ref["S"]
    pix_ties = near_half(ref["x_prop"]) | near_half(ref["y_prop"])
    assert np.all(pix_ties[bad]), np.flatnonzero(bad & ~pix_ties)[:10]
    if bad.any():
        return dict(pixel_ties=int(bad.sum()), cdf_ties=0)
    # normalised weights before resampling
    assert np.max(np.abs(got["w"] - ref["w"])) <= 1e-12
    assert abs(got["w"].sum() - 1.0) < 1e-12
    # estimate
    assert abs(est[0] - ref["est"][0]) <= 1e-9 and abs(est[1] - ref["est"][1]) <= 1e-9
    nties = 0
    if check_anc:
        mism = got["anc"] != ref["anc"]
        ties = anc_ties(ref, n)
        assert np.all(ties[mism]), np.flatnonzero(mism & ~ties)[:10]
        nties = int(mism.sum())
        ok = ~mism
        # the resampled state is the propagated position of the ancestor
        assert np.array_equal(got["x"][ok], ref["x"][ok]) or np.max(
            np.abs(got["x"][ok] - ref["x"][ok])) <= 1e-9
    assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])
    assert np.array_equal(got["y"], gs["y_prop"][got["anc"]])
    return dict(pixel_ties=0, cdf_ties=nties)


def check_resample_consistency(got, gs, n):
    """Properties of systematic resampling that hold in any precision: the
    state is the ancestors' propagated positions, ancestors are
    non-decreasing, and every particle's offspring count is floor or ceil of
    N w (one extra unit of slack for the reduced-precision distribution)."""
    a = got["anc"]
    assert a.min() >= 0 and a.max() < n
    assert np.all(np.diff(a) >= 0)
    assert np.array_equal(got["x"], gs["x_prop"][a])
    assert np.array_equal(got["y"], gs["y_prop"][a])
    counts = np.bincount(a, minlength=n)
    nw = n * got["w"]
    assert np.all(counts >= np.floor(nw) - 1) and np.all(counts <= np.ceil(nw) + 1)


def tv(a, b):
    return 0.5 * np.abs(a - b).sum()


def make_filter(dtype, n, W, H, r, x0, y0, drift=(1.0, -2.0), sigma=(5.0, 2.0), seed=0,
                stream_id=0, diagnostics=True, lik_norm=0, **variant):
    p = pf.make_params(n, W, H, dtype, radius=r, x0=x0, y0=y0, drift=drift, sigma=sigma,
                       seed=seed, stream_id=stream_id, diagnostics=diagnostics, lik_norm=lik_norm,
                       **variant)
    return pf.Filter(p)
