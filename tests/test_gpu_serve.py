"""GPU test of the serving path: streams pass through small slot pools (so
they queue and reuse slots re-initialised in place), and every stream's
estimates equal those of the same filter run alone on the same frames."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth
from paper_2308_00763_amd.serve import GpuPoolBackend, Scheduler, StreamRequest

pytestmark = pytest.mark.gpu


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def test_streams_through_pools_equal_alone_runs():
    rng = np.random.default_rng(8)
    clk = _Clock()
    be = GpuPoolBackend({"f16": {1024: 2, 4096: 1, 16384: 2}, "f32": {2048: 1, 16384: 2}})
    s = Scheduler(be, clock=clk, stall_timeout=10.0)
    reqs = []
    for sid in range(14):
        side = int(rng.choice([64, 128]))
        frames = int(rng.integers(4, 9))
        v = (int(rng.integers(-2, 3)), int(rng.integers(-2, 3)))
        start = (side // 2, side // 2)
        vid = pfsynth.moving_disk(side, side, frames, 5, start, v, float(rng.uniform(2, 6)),
                                  seed=500 + sid)
        dev = torch.from_numpy(vid.frames).to("cuda:0")
        dtype = "f16" if sid % 3 else "f32"
        n = int(rng.integers(300, 16000))
        p = pf.make_params(n, side, side, dtype, x0=start[0], y0=start[1], drift=v, seed=4,
                           stream_id=sid)
        r = StreamRequest(sid, 0.02 * sid, p, frames, 30.0, lambda i, d=dev: d[i])
        assert s.submit(r)
        reqs.append((r, dev))
    print("[serve] running", flush=True)
    summ = s.run(until=1e6, sleep=clk.sleep, poll=0.002)
    print(f"[serve] {summ}", flush=True)
    assert summ["streams"] == {"done": 14}
    waited = sum(1 for r in s.results.values() if r.admission_wait > 0)
    assert waited > 0  # the pools are too small for every stream at once
    for r, dev in reqs:
        f = pf.Filter(r.params)
        ests = []
        for i in range(1, r.n_frames):
            f.step(dev[i])
            ests.append(f.estimate())
        f.close()
        assert np.array_equal(np.array(ests), np.array(s.results[r.sid].estimates)), r.sid
    be.close()


def test_reinit_refuses_parameters_larger_than_the_share():
    b = pf.Batch([pf.make_params(2048, 64, 64, "f16"), pf.make_params(1024, 64, 64, "f16")])
    with pytest.raises(pf.PfError) as ei:
        b.reinit(1, pf.make_params(2048, 64, 64, "f16"))
    assert ei.value.code == pf.PF_ERR_WORKSPACE
    with pytest.raises(pf.PfError) as ei:
        b.reinit(0, pf.make_params(1000, 64, 64, "f32"))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    b.reinit(0, pf.make_params(1500, 64, 64, "f16", x0=10, y0=20))
    assert pf.pf_estimate(b.filter(0)) == (10.0, 20.0)
    assert b.export(0)["t"] == 0
    b.close()
