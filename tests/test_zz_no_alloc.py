"""The allocation-free step (pf_step_static_scratch) against pf_step.

A filter created with PF_FLAG_STATE_ONLY keeps only its state in its
workspace and steps through the library's static device scratch; its
estimates, particles, weights and ancestors must be bit-identical to pf_step
on a filter with the same parameters, frames and step count.  Two filters
in a row share the scratch, the second smaller than the first, so the
second call runs on what the first left in it.
"""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth

pytestmark = pytest.mark.gpu


def _pair(n, dtype, w, vid, steps):
    x0, y0 = vid.centres[0]
    kw = dict(radius=w.radius, x0=x0, y0=y0, drift=w.drift, sigma=w.sigma, seed=3, stream_id=11,
              diagnostics=True)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    a = pf.Filter(pf.make_params(n, w.width, w.height, dtype, **kw))
    b = pf.Filter(pf.make_params(n, w.width, w.height, dtype, state_only=True, **kw))
    assert b.workspace.numel() < a.workspace.numel()
    for t in range(1, steps + 1):
        print(f"[no-alloc] N={n} {dtype} step {t}", flush=True)
        pf.pf_step(a.handle, fr[t].data_ptr(), fr[t].stride(0))
        pf.pf_step_static_scratch(b.handle, fr[t].data_ptr(), fr[t].stride(0))
        assert a.estimate() == b.estimate(), t
        ea, eb = a.export(), b.export()
        for k in ("x", "y", "w", "anc", "t"):
            assert np.array_equal(ea[k], eb[k]), (t, k)
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f16", "f64"])
def test_static_scratch_step_equals_pf_step(dtype):
    w = pfsynth.WORKLOADS["disk1024_n1m"]
    vid = pfsynth.workload_video(w, frames=5)
    # first call: 2^20 particles (1024 tiles); then a smaller filter on the
    # same scratch (ragged last tile, one combine class down)
    _pair(1 << 20, dtype, w, vid, 4)
    _pair(70001, dtype, w, vid, 3)


def test_static_scratch_refusals():
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w, frames=2)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    a = pf.Filter(pf.make_params(1000, 128, 128, "f16", x0=64, y0=64))
    with pytest.raises(pf.PfError) as ei:
        pf.pf_step_static_scratch(a.handle, fr[1].data_ptr(), fr[1].stride(0))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    b = pf.Filter(pf.make_params(1000, 128, 128, "f16", x0=64, y0=64, state_only=True))
    with pytest.raises(pf.PfError) as ei:
        pf.pf_step(b.handle, fr[1].data_ptr(), fr[1].stride(0))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    with pytest.raises(pf.PfError):
        pf.pf_step_static_scratch(b.handle, fr[1].data_ptr(), 100)  # pitch < W
    b.step(fr[1])
    with pytest.raises(pf.PfError):
        b.export_step()  # no propagated positions kept
    assert np.all(np.isfinite(b.estimate()))
    a.close()
    b.close()
