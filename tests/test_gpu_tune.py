"""GPU test of the workgroup-size autotuner: it times every candidate, picks
the fastest, and a filter built with its flags runs the same step (FP64:
element-wise parity with the default filter's estimates)."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth
from paper_2308_00763_amd.tune import PASS_A_THREADS, PASS_C_THREADS, autotune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f16", "f64"])
def test_autotune_picks_a_measured_candidate(dtype):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    n = 100_000
    res = autotune(n, w.width, w.height, fr, dtype=dtype, x0=vid.centres[0][0],
                   y0=vid.centres[0][1], steps=8, warmup=2)
    print(f"[tune] {dtype}: {res}", flush=True)
    assert res["threads_a"] in PASS_A_THREADS and res["threads_c"] in PASS_C_THREADS
    assert set(res["table"]["pass_a"]) == set(PASS_A_THREADS)
    assert set(res["table"]["pass_c"]) == set(PASS_C_THREADS)
    assert res["pass_a_us"] == min(res["table"]["pass_a"].values())
    assert res["pass_c_us"] == min(res["table"]["pass_c"].values())
    tuned = pf.make_params(n, w.width, w.height, dtype, x0=vid.centres[0][0], y0=vid.centres[0][1])
    tuned.flags |= res["flags"]
    base = pf.make_params(n, w.width, w.height, dtype, x0=vid.centres[0][0], y0=vid.centres[0][1])
    ests = []
    for p in (base, tuned):
        f = pf.Filter(p)
        e = []
        for t in range(1, w.frames):
            f.step(fr[t])
            e.append(f.estimate())
        f.close()
        ests.append(np.array(e))
    tol = 1e-9 if dtype == "f64" else 0.05
    assert np.max(np.abs(ests[0] - ests[1])) <= tol
