"""GPU parity of Gumbel-max multinomial resampling (PF_FLAG_GUMBEL_MAX)
against the oracle, teacher-forced on the 128 px video.  FP64: ancestors
equal the oracle's except where the best and second-best scores of a slot lie
within 1e-9 of each other.  Reduced modes: the oracle run on the GPU's own
integer disk terms; where a slot's ancestor differs, the oracle's score of
the GPU's choice must be within the two scores' reduced-arithmetic error of
the oracle's best score.  A score L_j + G is formed in float from the top 24
bits of the word: its error is |G(u32) - G(u24)| (computed exactly from the
word) plus the float rounding of L = S / denom, of the two logarithms and of
the sum, at most GUMBEL_REL (1 + |L| + |G|) with GUMBEL_REL = 1e-5 (a few
2^-23 per operation, and v_log_f32's absolute accuracy where -ln u is tiny)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_00763_amd as pf
import pfsynth
from gpu_common import make_filter, near_half, oracle_params, oracle_step_parts

pytestmark = pytest.mark.gpu

GUMBEL_REL = 1e-5


def _score_error_bound(L, i, j, seed, stream_id, t):
    """The oracle's score of pair (slot i, particle j) and the bound on the
    reduced kernel's error in it."""
    key = [seed & 0xFFFFFFFF, (seed >> 32) ^ 0x47756D62]
    w = int(oracle.philox4x32_10([j // 4, i, t, stream_id], key)[j % 4])
    u32 = (w + 0.5) * 2.0 ** -32
    u24 = ((w >> 8) + 0.5) * 2.0 ** -24
    g32, g24 = -np.log(-np.log(u32)), -np.log(-np.log(u24))
    return L[j] + g32, abs(g32 - g24) + GUMBEL_REL * (1 + abs(L[j]) + abs(g24))


def _run(dtype, n, steps=2):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    f = make_filter(dtype, n, w.width, w.height, 5, x0, y0, seed=12, stream_id=3, gumbel_max=True)
    op = oracle_params(n, w.width, w.height, 5, seed=12, stream_id=3)
    nd = oracle.disk(5)[0].size
    x, y = np.full(n, x0), np.full(n, y0)
    for t in range(1, steps + 1):
        print(f"[gumbel] {dtype} n={n} step={t}", flush=True)
        f.load(x, y, t - 1)
        f.step(fr[t])
        got, gs, est = f.export(), f.export_step(), f.estimate()
        ref = oracle_step_parts(op, t, vid.frames[t], x, y)
        yield t, got, gs, est, ref, op, nd
        x, y = ref["x_prop"][got["anc"]], ref["y_prop"][got["anc"]]
    f.close()


@pytest.mark.parametrize("n", [1000, 1025, 4999])
def test_f64_gumbel_max_matches_the_oracle(n):
    for t, got, gs, est, ref, op, nd in _run("f64", n):
        bad = gs["disk_sum"].astype(np.int64) != ref["S"]
        assert np.all((near_half(ref["x_prop"]) | near_half(ref["y_prop"]))[bad])
        if bad.any():
            continue
        assert abs(est[0] - ref["est"][0]) <= 1e-9 and abs(est[1] - ref["est"][1]) <= 1e-9
        anc, margin = oracle.gumbel_max(ref["L"], op.seed, op.stream_id, t)
        mism = got["anc"] != anc
        assert np.all(margin[mism] <= 1e-9), np.flatnonzero(mism & (margin > 1e-9))[:10]
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_reduced_gumbel_max_follows_the_oracle_on_its_own_disk_terms(dtype):
    n = 3000
    for t, got, gs, est, ref, op, nd in _run(dtype, n):
        L = gs["disk_sum"].astype(np.float64) / (op.kappa * nd)
        anc, margin = oracle.gumbel_max(L, op.seed, op.stream_id, t)
        mism = np.flatnonzero(got["anc"] != anc)
        print(f"[gumbel] {dtype} step {t}: {mism.size} of {n} slots differ", flush=True)
        for i in mism:
            s_best, e_best = _score_error_bound(L, int(i), int(anc[i]), op.seed, op.stream_id, t)
            s_got, e_got = _score_error_bound(L, int(i), int(got["anc"][i]), op.seed, op.stream_id, t)
            assert s_best - s_got <= e_best + e_got, (i, s_best - s_got, e_best + e_got)
        assert np.array_equal(got["x"], gs["x_prop"][got["anc"]])


def test_gumbel_max_limits():
    with pytest.raises(pf.PfError):
        pf.pf_workspace_bytes(pf.make_params(65537, 128, 128, gumbel_max=True))
    with pytest.raises(pf.PfError):
        pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, gumbel_max=True, metropolis_steps=4))
    pf.pf_workspace_bytes(pf.make_params(65536, 128, 128, gumbel_max=True))
