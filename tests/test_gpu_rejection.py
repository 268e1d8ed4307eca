"""GPU parity of rejection resampling (PF_FLAG_REJECTION) against the
oracle's (or_rejection), teacher-forced on the 128 px video.

FP64: the propagation, disk sums and estimate as in the systematic step, and
every slot's ancestor equal to the oracle's except where one of its trials'
acceptance tests lies within 1e-12 of its threshold (the oracle's margin).
Reduced modes: the oracle run on the GPU's own integer disk terms; a slot may
differ only where one of its tests lies within the reduced arithmetic's
resolution of the threshold: the uniform is the top 24 bits of the word
(|u24 - u32| <= 2^-24) and exp2((S_c - S_max) beta) is formed in float (the
exponent carries at most |S_c - S_max| beta 2^-23 <= 24 * 2^-23 of error
wherever the threshold is above 2^-24, so the ratio's relative error is below
2.1e-6, plus one ulp of v_exp_f32): REDUCED_MARGIN = 2^-24 + 2.5e-6."""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_00763_amd as pf
import pfsynth
from gpu_common import make_filter, near_half, oracle_params, oracle_step_parts

pytestmark = pytest.mark.gpu

REDUCED_MARGIN = 2.0 ** -24 + 2.5e-6


def _run(dtype, n, cap, steps=3):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    f = make_filter(dtype, n, w.width, w.height, 5, x0, y0, seed=8, stream_id=4,
                    rejection_trials=cap)
    op = oracle_params(n, w.width, w.height, 5, seed=8, stream_id=4)
    nd = oracle.disk(5)[0].size
    x, y = np.full(n, x0), np.full(n, y0)
    for t in range(1, steps + 1):
        print(f"[rejection] {dtype} n={n} cap={cap} step={t}", flush=True)
        f.load(x, y, t - 1)
        f.step(fr[t])
        got, gs, est = f.export(), f.export_step(), f.estimate()
        ref = oracle_step_parts(op, t, vid.frames[t], x, y)
        yield t, got, gs, est, ref, op, nd
        x, y = ref["x_prop"][got["anc"]], ref["y_prop"][got["anc"]]
    f.close()


@pytest.mark.parametrize("n,cap", [(1000, 4096), (5000, 64), (70001, 1024)])
def test_f64_rejection_matches_the_oracle(n, cap):
    for t, got, gs, est, ref, op, nd in _run("f64", n, cap):
        assert np.max(np.abs(gs["x_prop"] - ref["x_prop"])) <= 1e-9
        bad = gs["disk_sum"].astype(np.int64) != ref["S"]
        assert np.all((near_half(ref["x_prop"]) | near_half(ref["y_prop"]))[bad])
        if bad.any():
            continue
        assert abs(est[0] - ref["est"][0]) <= 1e-9 and abs(est[1] - ref["est"][1]) <= 1e-9
        anc, margin, trials = oracle.rejection(ref["L"], cap, op.seed, op.stream_id, t)
        mism = got["anc"] != anc
        print(f"[rejection] f64 step {t}: mean trials {trials.mean():.1f}, capped {np.sum(trials == cap)}, "
              f"mismatches {mism.sum()}", flush=True)
        assert np.all(margin[mism] <= 1e-12), np.flatnonzero(mism & (margin > 1e-12))[:10]
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])
        assert np.array_equal(got["y"], gs["y_prop"][got["anc"]])


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_reduced_rejection_follows_the_oracle_on_its_own_disk_terms(dtype):
    n, cap = 20000, 4096
    for t, got, gs, est, ref, op, nd in _run(dtype, n, cap):
        L = gs["disk_sum"].astype(np.float64) / (op.kappa * nd)
        anc, margin, _ = oracle.rejection(L, cap, op.seed, op.stream_id, t)
        mism = got["anc"] != anc
        print(f"[rejection] {dtype} step {t}: {mism.sum()} slots differ, all within the margin "
              f"{np.all(margin[mism] <= REDUCED_MARGIN)}", flush=True)
        assert np.all(margin[mism] <= REDUCED_MARGIN), np.flatnonzero(mism & (margin > REDUCED_MARGIN))[:10]
        assert got["anc"].min() >= 0 and got["anc"].max() < n
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])


def test_rejection_parameters_are_checked():
    with pytest.raises(ValueError):
        pf.make_params(1000, 128, 128, rejection_trials=100)
    with pytest.raises(pf.PfError):
        pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, rejection_trials=64, gumbel_max=True))
    p = pf.make_params(1000, 128, 128, rejection_trials=64 * 255)
    # the disk terms of every particle (the systematic filter's own workspace
    # holds the deferred-resampling buffers instead: compare member layouts)
    assert pf.pf_member_bytes(p) > pf.pf_member_bytes(pf.make_params(1000, 128, 128))
