"""GPU parity of Metropolis resampling (PF_FLAG_METROPOLIS) against the
oracle's chain: teacher-forced steps on the 128 px video.  FP64: the
propagation, disk sums, weights and estimate as in the systematic step, and
every slot's ancestor equal to the oracle's except where one of the chain's
comparisons lies within 1e-12 of its threshold.  Reduced modes: the oracle's
chain run on the GPU's own integer disk terms; a slot may differ only where
one of its chain's comparisons lies within the reduced arithmetic's
resolution of its threshold: the uniform is the top 24 bits of the word
(|u24 - u32| <= 2^-24) and exp2((S_i - S_k) beta) is formed in float (the
exponent carries at most |S_i - S_k| beta 2^-23 <= 24 * 2^-23 of error
wherever the threshold is above 2^-24, so the ratio's relative error is below
2.1e-6, plus one ulp of v_exp_f32): REDUCED_MARGIN = 2^-24 + 2.5e-6."""
import numpy as np
import pytest
import torch

import oracle
import pfsynth
from gpu_common import make_filter, near_half, oracle_params, oracle_step_parts

pytestmark = pytest.mark.gpu

REDUCED_MARGIN = 2.0 ** -24 + 2.5e-6


def _run(dtype, n, B, steps=3):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    f = make_filter(dtype, n, w.width, w.height, 5, x0, y0, seed=6, stream_id=2,
                    metropolis_steps=B)
    op = oracle_params(n, w.width, w.height, 5, seed=6, stream_id=2)
    nd = oracle.disk(5)[0].size
    x, y = np.full(n, x0), np.full(n, y0)
    for t in range(1, steps + 1):
        print(f"[metropolis] {dtype} n={n} B={B} step={t}", flush=True)
        f.load(x, y, t - 1)
        f.step(fr[t])
        got, gs, est = f.export(), f.export_step(), f.estimate()
        ref = oracle_step_parts(op, t, vid.frames[t], x, y)
        yield t, got, gs, est, ref, op, nd
        x, y = ref["x_prop"][got["anc"]], ref["y_prop"][got["anc"]]
    f.close()


@pytest.mark.parametrize("n,B", [(1000, 32), (5000, 7), (70001, 64)])
def test_f64_metropolis_matches_the_oracle_chain(n, B):
    for t, got, gs, est, ref, op, nd in _run("f64", n, B):
        assert np.max(np.abs(gs["x_prop"] - ref["x_prop"])) <= 1e-9
        bad = gs["disk_sum"].astype(np.int64) != ref["S"]
        ties = near_half(ref["x_prop"]) | near_half(ref["y_prop"])
        assert np.all(ties[bad])
        if bad.any():
            continue
        assert np.max(np.abs(got["w"] - ref["w"])) <= 1e-12
        assert abs(est[0] - ref["est"][0]) <= 1e-9 and abs(est[1] - ref["est"][1]) <= 1e-9
        anc, margin = oracle.metropolis(ref["L"], B, op.seed, op.stream_id, t)
        mism = got["anc"] != anc
        assert np.all(margin[mism] <= 1e-12), np.flatnonzero(mism & (margin > 1e-12))[:10]
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])
        assert np.array_equal(got["y"], gs["y_prop"][got["anc"]])


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_reduced_metropolis_follows_the_oracle_chain_on_its_own_disk_terms(dtype):
    n, B = 20000, 32
    for t, got, gs, est, ref, op, nd in _run(dtype, n, B):
        L = gs["disk_sum"].astype(np.float64) / (op.kappa * nd)
        anc, margin = oracle.metropolis(L, B, op.seed, op.stream_id, t)
        mism = got["anc"] != anc
        print(f"[metropolis] {dtype} step {t}: {mism.sum()} of {n} slots differ", flush=True)
        assert np.all(margin[mism] <= REDUCED_MARGIN), np.flatnonzero(mism & (margin > REDUCED_MARGIN))[:10]
        assert got["anc"].min() >= 0 and got["anc"].max() < n
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])


def test_metropolis_steps_are_checked():
    import paper_2308_00763_amd as pf
    with pytest.raises(ValueError):
        pf.make_params(1000, 128, 128, metropolis_steps=256)
    with pytest.raises(pf.PfError):
        pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, metropolis_steps=8,
                                             naive_resample=True))
