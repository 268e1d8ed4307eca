"""GPU tests of the implementation variants (the straightforward likelihood
and resampler, and other workgroup sizes): the same step as the default, so
FP64 keeps element-wise parity with the oracle, the reduced modes resample as
the FP64 step of their own disk sums does (within the mode's resolution, which
the straightforward resampler's float distribution widens), and variants that
do not change the arithmetic give bit-identical results."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth
from gpu_common import (check_reduced_step, compare_f64_step, make_filter, oracle_params,
                        oracle_step_parts, tv)

pytestmark = pytest.mark.gpu

VARIANTS = [
    dict(naive_likelihood=True),
    dict(naive_resample=True),
    dict(naive_resample=True, threads_c=64),
    dict(naive_resample=True, threads_c=1024),
    dict(threads_a=128),
    dict(threads_a=512),
    dict(threads_c=64),
    dict(threads_c=128),
    dict(threads_c=256),
    dict(threads_c=512),
    dict(threads_c=1024),
    dict(naive_likelihood=True, naive_resample=True, threads_a=128, threads_c=128),
]


def _vid():
    w = pfsynth.WORKLOADS["disk128_n1000"]
    return w, pfsynth.workload_video(w)


def _teacher_forced(dtype, n, vid, steps, **variant):
    T, H, W = vid.frames.shape
    x0, y0 = vid.centres[0]
    f = make_filter(dtype, n, W, H, 5, x0, y0, **variant)
    op = oracle_params(n, W, H, 5)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x, y = np.full(n, x0), np.full(n, y0)
    out = []
    for t in range(1, steps + 1):
        print(f"[variant] {dtype} n={n} {variant} step={t}", flush=True)
        f.load(x, y, t - 1)
        f.step(fr[t])
        got, gs, est = f.export(), f.export_step(), f.estimate()
        ref = oracle_step_parts(op, t, vid.frames[t], x, y)
        out.append((got, gs, est, ref))
        x, y = ref["x"], ref["y"]
    f.close()
    return out


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "-".join(f"{k}={x}" for k, x in v.items()))
@pytest.mark.parametrize("n", [1025, 5000])
def test_f64_variant_matches_oracle(variant, n):
    _, vid = _vid()
    for got, gs, est, ref in _teacher_forced("f64", n, vid, 3, **variant):
        compare_f64_step(got, gs, est, ref, n)


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "-".join(f"{k}={x}" for k, x in v.items()))
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_reduced_variant_resamples_as_fp64_does(variant, dtype):
    _, vid = _vid()
    n = 5000
    for got, gs, est, ref in _teacher_forced(dtype, n, vid, 3, **variant):
        check_reduced_step(got, gs, est, ref["u0"], ref["denom"], n, dtype,
                           naive=bool(variant.get("naive_resample")))
        assert tv(got["w"], ref["w"]) <= 0.1


def _free_run(dtype, n, **variant):
    w, vid = _vid()
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    f = make_filter(dtype, n, w.width, w.height, 5, *vid.centres[0], **variant)
    ests = []
    for t in range(1, w.frames):
        f.step(fr[t])
        ests.append(f.estimate())
    got = f.export()
    f.close()
    return np.array(ests), got


@pytest.mark.parametrize("variant", [dict(naive_likelihood=True), dict(threads_c=64),
                                     dict(threads_c=128), dict(threads_c=256), dict(threads_c=512),
                                     dict(threads_c=1024)],
                         ids=lambda v: "-".join(f"{k}={x}" for k, x in v.items()))
@pytest.mark.parametrize("dtype", ["f64", "f16"])
def test_variants_with_the_same_arithmetic_are_bit_identical(variant, dtype):
    n = 70001
    e0, g0 = _free_run(dtype, n)
    e1, g1 = _free_run(dtype, n, **variant)
    assert np.array_equal(e0, e1)
    for key in ("x", "y", "w", "anc"):
        assert np.array_equal(g0[key], g1[key]), key


@pytest.mark.parametrize("n", [5000, 70001, (1 << 20) + 3])
def test_unpacked_half_propagation_is_bit_identical(n):
    # the paper's straightforward half step propagates one particle at a
    # time; each scalar operation rounds as its lane of the packed one does
    e0, g0 = _free_run("f16", n)
    e1, g1 = _free_run("f16", n, naive_half=True)
    assert np.array_equal(e0, e1)
    for key in ("x", "y", "w", "anc"):
        assert np.array_equal(g0[key], g1[key]), key


def test_naive_half_step_resamples_as_fp64_does():
    # unpacked half with the straightforward resampler (a division per
    # particle and casts): the step the paper's optimisation starts from
    w, vid = _vid()
    for got, gs, est, ref in _teacher_forced("f16", 5000, vid, 3, naive_half=True, naive_resample=True):
        check_reduced_step(got, gs, est, ref["u0"], ref["denom"], 5000, "f16", naive=True)


@pytest.mark.parametrize("threads_c", [64, 1024])
@pytest.mark.parametrize("dtype", ["f64", "f16"])
def test_streaming_pass_c_sizes_are_bit_identical_over_many_tiles(threads_c, dtype):
    # 4097 tiles: each resident pass-C workgroup streams several of them (a
    # grid of a few hundred 1024-thread workgroups, or of a few thousand
    # 64-thread ones), and the last tile is ragged
    n = (1 << 22) + 77
    e0, g0 = _free_run(dtype, n)
    e1, g1 = _free_run(dtype, n, threads_c=threads_c)
    assert np.array_equal(e0, e1)
    for key in ("x", "y", "w", "anc"):
        assert np.array_equal(g0[key], g1[key]), key


def test_variant_flags_are_checked():
    for bad in (dict(threads_a=64), dict(threads_a=1024)):
        with pytest.raises(pf.PfError):
            pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, **bad))
    with pytest.raises(ValueError):
        pf.make_params(1000, 128, 128, threads_c=96)
    with pytest.raises(pf.PfError):
        pf.Batch([pf.make_params(1000, 128, 128, "f16", naive_resample=True)])
    for bad in (dict(dtype="f32", naive_half=True), dict(dtype="f16", naive_half=True, threads_a=128)):
        with pytest.raises(pf.PfError):
            pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, **bad))
    # the normalised distribution (member layouts: the systematic filter's own
    # workspace holds the deferred-resampling buffers instead)
    base = pf.pf_member_bytes(pf.make_params(1 << 20, 128, 128, "f16"))
    naive = pf.pf_member_bytes(pf.make_params(1 << 20, 128, 128, "f16", naive_resample=True))
    assert naive - base >= 4 << 20
