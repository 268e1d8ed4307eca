"""GPU test of the serving path: streams pass through small slot pools (so
they queue and reuse slots re-initialised in place), and every stream's
estimates equal those of the same filter run alone on the same frames."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth
from paper_2308_00763_amd.serve import FrameSeq, GpuByteBackend, GpuPoolBackend, Scheduler, StreamRequest

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


def _stream_requests(n_streams, seed):
    rng = np.random.default_rng(seed)
    out = []
    for sid in range(n_streams):
        side = int(rng.choice([64, 128]))
        frames = int(rng.integers(4, 9))
        v = (int(rng.integers(-2, 3)), int(rng.integers(-2, 3)))
        start = (side // 2, side // 2)
        vid = pfsynth.moving_disk(side, side, frames, 5, start, v, float(rng.uniform(2, 6)), seed=700 + sid)
        dev = torch.from_numpy(vid.frames).to("cuda:0")
        dtype = "f16" if sid % 3 else "f32"
        n = int(np.exp(rng.uniform(np.log(300), np.log(60000))))
        p = pf.make_params(n, side, side, dtype, x0=start[0], y0=start[1], drift=v, seed=4, stream_id=sid)
        out.append((StreamRequest(sid, 0.02 * sid, p, frames, 30.0, lambda i, d=dev: d[i]), dev))
    return out


@pytest.mark.parametrize("plan_factor", [2.0, 0.5])
def test_streams_through_a_byte_budget_equal_alone_runs(plan_factor):
    # budgets that hold a few streams at a time: admission waits for bytes;
    # with half the arena's worth of tiles in the plan, idle members' stale
    # tiles must be parked to admit new streams
    clk = _Clock()
    budgets = {"f16": 3 * pf.pf_member_bytes(pf.make_params(60000, 64, 64, "f16")),
               "f32": 2 * pf.pf_member_bytes(pf.make_params(60000, 64, 64, "f32"))}
    be = GpuByteBackend(budgets, {"f16": 6, "f32": 4}, plan_factor=plan_factor)
    s = Scheduler(be, clock=clk, stall_timeout=10.0)
    reqs = _stream_requests(16, seed=12)
    for r, _ in reqs:
        assert s.submit(r)
    print("[serve] byte budget running", flush=True)
    summ = s.run(until=1e6, sleep=clk.sleep, poll=0.002)
    print(f"[serve] {summ}", flush=True)
    assert summ["streams"] == {"done": 16}
    assert sum(1 for r in s.results.values() if r.admission_wait > 0) > 0
    assert be.in_use() == 0 and all(a.starts == [0] for a in be.arenas.values())
    assert summ["hbm_high_water_bytes"] <= sum(budgets.values())
    for dt in be.batches:  # the members' tiles as the backend counts them stay within the plan
        assert be.tiles_used[dt] == sum(be.cur_tiles[dt]) <= be.tiles_cap[dt]
    for r, dev in reqs:
        f = pf.Filter(r.params)
        ests = []
        for i in range(1, r.n_frames):
            f.step(dev[i])
            ests.append(f.estimate())
        f.close()
        assert np.array_equal(np.array(ests), np.array(s.results[r.sid].estimates)), r.sid
    be.close()


def test_a_stream_larger_than_the_budget_is_rejected_at_submission():
    be = GpuByteBackend({"f16": 1 << 20}, {"f16": 2})
    s = Scheduler(be, clock=_Clock())
    big = pf.make_params(1 << 20, 64, 64, "f16")
    assert not s.submit(StreamRequest(0, 0.0, big, 3, 30.0, lambda i: None))
    assert s.results[0].status == "rejected" and "budget" in s.results[0].reason
    be.close()


def test_rebind_to_caller_shares_and_its_refusals():
    T = 6
    (r0, dev0), (r1, dev1) = _stream_requests(2, seed=4)
    p0 = pf.make_params(50000, r0.params.width, r0.params.height, "f16", x0=r0.params.x0, y0=r0.params.y0,
                        drift=(r0.params.drift_x, r0.params.drift_y), seed=4, stream_id=0)
    tiny = pf.make_params(1, 64, 64, "f16")
    # plan capacity: two one-tile members plus the 49 tiles of p0
    b = pf.Batch([tiny, tiny], max_tiles=2 + 48)
    need = pf.pf_member_bytes(p0)
    share = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    base = share.data_ptr()
    with pytest.raises(pf.PfError) as ei:   # misaligned
        b.rebind(0, p0, base + 8, need)
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    with pytest.raises(pf.PfError) as ei:   # share too small
        b.rebind(0, p0, base, need - 256)
    assert ei.value.code == pf.PF_ERR_WORKSPACE
    b.rebind(0, p0, base, need)
    # a second 49-tile member would exceed the plan: refused, nothing changes
    other = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(pf.PfError) as ei:
        b.rebind(1, p0, other.data_ptr(), need)
    assert ei.value.code == pf.PF_ERR_WORKSPACE
    frames = dev0
    for t in range(1, min(T, r0.n_frames)):
        b.step([frames[t], None], np.array([1, 0], np.uint8))
    est_a, got_a = [], None
    f = pf.Filter(p0)
    for t in range(1, min(T, r0.n_frames)):
        f.step(frames[t])
        est_a.append(f.estimate())
    got_a = f.export()
    f.close()
    assert np.array_equal(np.array(est_a[-1]), b.estimates()[0])
    got_b = b.export(0)
    assert np.array_equal(got_a["x"], got_b["x"]) and np.array_equal(got_a["y"], got_b["y"])
    # reinit after a rebind reuses the caller's share (bytes of the rebind)
    b.reinit(0, pf.make_params(40000, 64, 64, "f16", x0=5, y0=6))
    assert pf.pf_estimate(b.filter(0)) == (5.0, 6.0)
    b.close()


def test_idle_members_are_parked_when_the_plan_is_full():
    # three handles, a budget and a plan for two 20000-particle streams (20
    # tiles each): after A and B finish their members keep 20 stale tiles
    # each, so admitting C (30000 particles, 30 tiles) on one of them must
    # park the other; C then runs exactly as it does alone
    T = 5
    reqs = _stream_requests(3, seed=21)
    ps = []
    for sid, (r, dev) in enumerate(reqs):
        p = pf.make_params(30000 if sid == 2 else 20000, r.params.width, r.params.height, "f16",
                           x0=r.params.x0, y0=r.params.y0, drift=(r.params.drift_x, r.params.drift_y),
                           seed=4, stream_id=sid)
        ps.append((StreamRequest(sid, 0.0, p, T, 30.0, r.frame), dev))
    budget = 2 * pf.pf_member_bytes(ps[0][0].params)
    be = GpuByteBackend({"f16": budget}, {"f16": 3}, plan_factor=1.0)
    assert 41 <= be.tiles_cap["f16"] < 51
    sa = be.try_admit(ps[0][0])
    sb = be.try_admit(ps[1][0])
    assert sa is not None and sb is not None
    assert be.try_admit(ps[2][0]) is None          # the bytes are taken
    be.release(sa)
    be.release(sb)
    assert be.parked == 0
    sc = be.try_admit(ps[2][0])
    assert sc is not None and be.parked >= 1
    assert be.tiles_used["f16"] == sum(be.cur_tiles["f16"]) <= be.tiles_cap["f16"]
    r, dev = ps[2]
    ests = []
    for t in range(1, T):
        assert not be.step([(sc, dev[t])])
        ests.append(be.estimates([sc])[0])
    f = pf.Filter(r.params)
    alone = []
    for t in range(1, T):
        f.step(dev[t])
        alone.append(f.estimate())
    f.close()
    assert np.array_equal(np.array(ests), np.array(alone))
    be.close()


def test_frameseq_streams_through_the_byte_backend_equal_alone_runs():
    # FrameSeq sources: the scheduler steps these streams from its columns
    # through the backend's array calls
    clk = _Clock()
    budgets = {"f16": 3 * pf.pf_member_bytes(pf.make_params(60000, 64, 64, "f16")),
               "f32": 2 * pf.pf_member_bytes(pf.make_params(60000, 64, 64, "f32"))}
    be = GpuByteBackend(budgets, {"f16": 6, "f32": 4})
    s = Scheduler(be, clock=clk, stall_timeout=10.0)
    reqs = _stream_requests(12, seed=31)
    for r, dev in reqs:
        r.frame = FrameSeq(dev.data_ptr(), dev.stride(0), dev.stride(1))
        assert s.submit(r)
    print("[serve] frameseq running", flush=True)
    summ = s.run(until=1e6, sleep=clk.sleep, poll=0.002)
    print(f"[serve] {summ}", flush=True)
    assert summ["streams"] == {"done": 12}
    assert not s.due and not s.cols.used.any()
    for r, dev in reqs:
        f = pf.Filter(r.params)
        ests = []
        for i in range(1, r.n_frames):
            f.step(dev[i])
            ests.append(f.estimate())
        f.close()
        assert np.array_equal(np.array(ests), np.array(s.results[r.sid].estimates)), r.sid
    be.close()
