"""GPU tests at the largest particle count the library accepts (N = 2^28:
262 144 tiles, the grouped combine's full 256 groups, the streaming pass C
at 128 tiles per workgroup): two steps in FP64 and FP16 on the 1024x1024
video; the estimates must follow the disk's centre and agree between modes.
(The oracle cannot run at this size; the step's parts are checked against it
at every smaller size.)"""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth

pytestmark = pytest.mark.gpu

N_MAX = 1 << 28


def _run(dtype, fr, w, x0, y0, steps):
    p = pf.make_params(N_MAX, w.width, w.height, dtype, radius=w.radius, x0=x0, y0=y0,
                       drift=w.drift, sigma=w.sigma, seed=w.filter_seed)
    f = pf.Filter(p)
    est = []
    for t in range(1, steps + 1):
        print(f"[limits] {dtype} N=2^28 step {t}", flush=True)
        f.step(fr[t])
        est.append(f.estimate())
    f.close()
    del f
    torch.cuda.empty_cache()
    return np.array(est)


def test_largest_particle_count():
    w = pfsynth.WORKLOADS["disk1024_n1m"]
    vid = pfsynth.workload_video(w, frames=3)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    x0, y0 = vid.centres[0]
    e64 = _run("f64", fr, w, x0, y0, 2)
    e16 = _run("f16", fr, w, x0, y0, 2)
    truth = np.array(vid.centres[1:3])
    assert np.all(np.isfinite(e64)) and np.all(np.isfinite(e16))
    # 2^28 particles: the estimate is the posterior mean to a few thousandths
    # of a pixel, within the pixel noise of the disk's true centre
    assert np.max(np.hypot(*(e64 - truth).T)) < 0.5, (e64, truth)
    assert np.max(np.hypot(*(e16 - e64).T)) < 0.05, (e16, e64)
