"""GPU test of HIP graph capture of pf_step: a filter whose step was captured
once and replayed on a refilled frame buffer, with eager copies and
synchronisations between the replays, gives every estimate and the final
state bit-identical to the same filter stepped eagerly."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,n", [("f64", 5000), ("f16", 70001), ("bf16", (1 << 22) + 1)])
def test_replayed_graph_equals_eager_steps(dtype, n):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    p = pf.make_params(n, w.width, w.height, dtype, x0=x0, y0=y0, seed=2, diagnostics=True)

    eager = pf.Filter(p)
    e_est = []
    for t in range(1, w.frames):
        eager.step(fr[t])
        e_est.append(eager.estimate())
    e_got = eager.export()
    eager.close()

    side = torch.cuda.Stream()
    f = pf.Filter(p, stream=side)
    static = torch.zeros((w.height, w.width), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        pf.pf_step(f.handle, static.data_ptr(), w.width)
    torch.cuda.synchronize()
    g_est = []
    for t in range(1, w.frames):
        print(f"[graph] {dtype} n={n} replay {t}", flush=True)
        static.copy_(fr[t])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        g_est.append(f.estimate())
    g_got = f.export()
    f.close()
    assert g_got["t"] == e_got["t"] == w.frames - 1
    assert np.array_equal(np.array(g_est), np.array(e_est))
    for key in ("x", "y", "w", "anc"):
        assert np.array_equal(g_got[key], e_got[key]), key
