"""Shared helpers of the GPU parity tests: teacher-forced stepping of the HIP
filter against the FP64 CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2308_00763_amd as pf

PIX_TIE = 1e-9   # a coordinate this close to a half-integer may round either way
CDF_TIE = 1e-12  # a stratum point this close to a CDF value may fall either side
U24 = 2.0 ** -24  # unit roundoff of float


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
    ref.update(x_prop=xp, y_prop=yp, L=L, u0=u0, denom=denom,
               S=np.rint(L * denom).astype(np.int64))
    return ref


def near_half(v, tol=PIX_TIE):
    return np.abs((v - 0.5) - np.round(v - 0.5)) < tol


def slot_coords(ref, n):
    """y_i = N C_i - u0: particle i ends the strata j with j <= y_i, so the
    ancestor of slot j is the first i with y_i >= j (the oracle's rule
    C_i >= (j + u0) / N written in slot units)."""
    return n * ref["cdf"] - ref["u0"]


def boundary_gap(y, anc_ref, anc_got, n):
    """For every slot, the distance (in slots) between the stratum point and
    the distribution boundary that separates the two ancestors: for an
    ancestor past the reference's (b > a) that is y_{b-1} - j, for one before
    it (b < a) j - y_b.  Zero where the ancestors agree."""
    j = np.arange(n, dtype=np.float64)
    a = anc_ref.astype(np.int64)
    b = anc_got.astype(np.int64)
    i = np.where(b > a, b - 1, b)
    gap = np.abs(y[np.clip(i, 0, n - 1)] - j)
    return np.where(a == b, 0.0, gap), i


def anc_ties(ref, n, got_anc=None):
    """Slots whose stratum point lies within CDF_TIE (in units of the
    distribution) of the boundary between the oracle's ancestor and the
    GPU's (either side may be chosen).  Without got_anc, the boundaries on
    both sides of the oracle's ancestor."""
    if got_anc is not None:
        gap, _ = boundary_gap(slot_coords(ref, n), ref["anc"], got_anc, n)
        return gap <= CDF_TIE * n
    j = np.arange(n)
    u = (j + ref["u0"]) / n
    C = ref["cdf"]
    a = ref["anc"]
    lo = np.where(a > 0, C[np.maximum(a - 1, 0)], -1.0)
    return (np.abs(u - C[a]) <= CDF_TIE) | (np.abs(u - lo) <= CDF_TIE)


def fp64_step_of(gs, u0, denom):
    """The FP64 weighting, normalisation, estimate and systematic resampling
    (the oracle's) of the GPU's own step: its integer disk sums and its
    propagated positions."""
    L = gs["disk_sum"].astype(np.float64) / denom
    ref = oracle.reweight_resample(L, gs["x_prop"], gs["y_prop"], u0)
    ref.update(L=L, u0=u0, denom=denom)
    return ref


def compare_f64_step(got, gs, est, ref, n, check_anc=True):
    """Element-wise parity of one teacher-forced FP64 step; returns counts of
    the mismatches that the tie rules excuse.

    Disk sums may differ only where a propagated coordinate lies within
    PIX_TIE of a rounding boundary; on such a step the rest of the step is
    compared with the oracle's weighting and resampling of the GPU's own disk
    sums, so every particle is still checked."""
    # propagation: same random stream, libm-level differences only
    assert np.max(np.abs(gs["x_prop"] - ref["x_prop"])) <= 1e-9
    assert np.max(np.abs(gs["y_prop"] - ref["y_prop"])) <= 1e-9
    # disk sums: integers, exact unless the pixel rounding is a tie
    bad = gs["disk_sum"].astype(np.int64) != ref["S"]
    pix_ties = near_half(ref["x_prop"]) | near_half(ref["y_prop"])
    assert np.all(pix_ties[bad]), np.flatnonzero(bad & ~pix_ties)[:10]
    npix = int(bad.sum())
    if npix:
        ref = fp64_step_of(gs, ref["u0"], ref["denom"])
    # normalised weights before resampling
    assert np.max(np.abs(got["w"] - ref["w"])) <= 1e-12
    assert abs(got["w"].sum() - 1.0) < 1e-12
    # estimate
    assert abs(est[0] - ref["est"][0]) <= 1e-9 and abs(est[1] - ref["est"][1]) <= 1e-9
    nties = 0
    if check_anc:
        mism = got["anc"] != ref["anc"]
        ties = anc_ties(ref, n, got["anc"])
        assert np.all(ties[mism]), np.flatnonzero(mism & ~ties)[:10]
        nties = int(mism.sum())
        ok = ~mism
        # the resampled state is the propagated position of the ancestor
        assert np.max(np.abs(got["x"][ok] - ref["x"][ok]), initial=0.0) <= 1e-9
        assert np.max(np.abs(got["y"][ok] - ref["y"][ok]), initial=0.0) <= 1e-9
    assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])
    assert np.array_equal(got["y"], gs["y_prop"][got["anc"]])
    return dict(pixel_ties=npix, cdf_ties=nties)


# ---------------------------------------------------------------------------
# Reduced modes (FP32, FP16, BF16): the ancestors must be the FP64 systematic
# resample of the step's own disk sums except where the stratum point lies
# within the mode's distribution resolution of the boundary between the two
# ancestors.  The resolution (in slots) bounds the difference between the
# mode's slot coordinate N P_i / Z - u0 and the FP64 one; its terms follow the
# mode's arithmetic:
#   weights   w_k f_t = 2^(d_k beta_f) 2^(d_t beta_f) with beta_f the float of
#             log2(e) / denom and d the integer differences of disk sums: a
#             relative error of at most |L_k - M| 2^-23 + 2^-21 (argument
#             roundings and two exponentials of 2 ulp); exactly 1 where the
#             disk sum is the step's maximum; weights below 2^-100 may be
#             lost entirely (flushed);
#   sums      the tile-local prefix sums in float: at most 16 roundings along
#             any path, a relative error of gamma_16 = 2^-20 of the mass
#             summed -- zero in tiles whose weights are all exactly one or
#             below 2^-60 (integer partial sums are exact), so only tiles
#             holding other weights contribute;
#   normaliser the errors above in Z move every coordinate in proportion to
#             C_i;
#   slot map  the two-float tile offsets, N / Z and u0 (2^-40 N), then the
#             float base fraction, the float scale and the fused
#             multiply-add of the particle's offset from the tile base
#             (2^-22 (|y_loc| + 1)).
# The straightforward resampler (normalised float distribution and float
# stratum points) adds 2^-22 (y_i + 2).

GAMMA16 = 2.0 ** -20


def reduced_slot_resolution(ref, n, naive=False):
    """Per particle, the bound on |y_mode - y_64| in slots (see above);
    `ref` is the FP64 step of the mode's own disk sums (fp64_step_of)."""
    L = ref["L"]
    M = L.max()
    wh = np.exp(L - M)                      # weights relative to the maximum
    top = L == M
    e = np.where(top, 0.0, wh * (np.abs(L - M) * 2.0 ** -23 + 2.0 ** -21))
    e = np.where(wh < 2.0 ** -100, np.maximum(e, wh), e)
    inexact = ~top & (wh >= 2.0 ** -60)
    npad = ((n + 1023) // 1024) * 1024
    tile_inexact = np.zeros(npad, dtype=bool)
    tile_inexact[:n] = inexact
    tile_inexact = tile_inexact.reshape(-1, 1024).any(axis=1)
    mass_in = np.where(np.repeat(tile_inexact, 1024)[:n], wh, 0.0)
    Z = wh.sum()
    Ecum = np.cumsum(e)
    Pin = np.cumsum(mass_in)
    C = ref["cdf"]
    y = slot_coords(ref, n)
    # slot coordinate of each tile's base (the end of the tile before)
    first = np.arange(n) - (np.arange(n) % 1024)
    base = np.where(first > 0, y[np.maximum(first - 1, 0)], -ref["u0"])
    y_loc = y - np.floor(base)
    tau = ((n / Z) * (Ecum + Ecum[-1] * C) + GAMMA16 * (n / Z) * (Pin + Pin[-1] * C)
           + 2.0 ** -22 * (np.abs(y_loc) + 1.0) + 2.0 ** -40 * n)
    if naive:
        tau = tau + 2.0 ** -22 * (np.abs(y) + 2.0)
    return tau, dict(Z=Z, E_tot=float(Ecum[-1]), P_inexact=float(Pin[-1]),
                     inexact_particles=int(inexact.sum()))


def check_reduced_step(got, gs, est, u0, denom, n, dtype, naive=False):
    """Strict parity of one reduced-precision step against the FP64 step of
    its own disk sums and propagated positions: every ancestor equals the
    FP64 systematic resample except where the stratum point lies within the
    mode's resolution of the boundary; normalised weights within the mode's
    rounding; estimate close; the state is the ancestors' propagated
    positions.  Returns the number of excused slots and the resolution
    summary."""
    a = got["anc"]
    assert a.min() >= 0 and a.max() < n
    assert np.all(np.diff(a) >= 0)
    assert np.array_equal(got["x"], gs["x_prop"][a])
    assert np.array_equal(got["y"], gs["y_prop"][a])
    ref = fp64_step_of(gs, u0, denom)
    tau, info = reduced_slot_resolution(ref, n, naive=naive)
    y = slot_coords(ref, n)
    gap, i = boundary_gap(y, ref["anc"], a, n)
    mism = ref["anc"] != a
    excused = gap <= tau[np.clip(i, 0, n - 1)]
    bad = mism & ~excused
    assert not bad.any(), (
        f"{int(bad.sum())} slots off the FP64 resample beyond the resolution; first "
        f"{np.flatnonzero(bad)[:8]}, gap {gap[bad][:8]}, tau {tau[np.clip(i, 0, n - 1)][bad][:8]}")
    # normalised weights: the errors above relative to Z, plus the float
    # division of the exported weights
    rel = (info["E_tot"] + GAMMA16 * info["P_inexact"]) / info["Z"]
    d = tv(got["w"], ref["w"])
    assert d <= 2.0 * rel + 2.0 ** -20, (d, rel)
    assert abs(got["w"].sum() - 1.0) <= 1e-5
    # estimate: same weights and positions; BF16 estimates from the float
    # positions before they are rounded to bfloat16 for storage
    tol = 0.02 if dtype == "bf16" else 1e-3
    assert abs(est[0] - ref["est"][0]) <= tol and abs(est[1] - ref["est"][1]) <= tol, (est, ref["est"])
    info.update(excused=int(mism.sum()), tv=d)
    return info


def check_resample_consistency(got, gs, n):
    """Properties of systematic resampling that hold in any precision and
    for any offset: the state is the ancestors' propagated positions and
    ancestors are non-decreasing (used where the resampler is not the
    systematic one of a known offset)."""
    a = got["anc"]
    assert a.min() >= 0 and a.max() < n
    assert np.all(np.diff(a) >= 0)
    assert np.array_equal(got["x"], gs["x_prop"][a])
    assert np.array_equal(got["y"], gs["y_prop"][a])


def tv(a, b):
    return 0.5 * np.abs(a - b).sum()


def make_filter(dtype, n, W, H, r, x0, y0, drift=(1.0, -2.0), sigma=(5.0, 2.0), seed=0,
                stream_id=0, diagnostics=True, lik_norm=0, **variant):
    p = pf.make_params(n, W, H, dtype, radius=r, x0=x0, y0=y0, drift=drift, sigma=sigma,
                       seed=seed, stream_id=stream_id, diagnostics=diagnostics, lik_norm=lik_norm,
                       **variant)
    return pf.Filter(p)
