"""CPU tests of the continuous-batching scheduler with an oracle-backed fake
backend on a virtual clock: admission against a slot budget, rejection,
stall eviction, failure isolation, frame order and latency accounting."""
import numpy as np
import pytest

import oracle
import paper_2308_00763_amd as pf
import pfsynth
from paper_2308_00763_amd.serve import Scheduler, StreamRequest, plan_pool, slot_classes
from serve_fake import FakeBackend, VirtualClock

SIDE = 64


def _stream(sid, arrival, n=300, frames=6, fps=10.0, stall_from=None, seed=0):
    v = (1 + sid % 2, -1)
    vid = pfsynth.moving_disk(SIDE, SIDE, frames, 5, (30, 34), v, 2.0, seed=100 + sid)
    p = pf.make_params(n, SIDE, SIDE, "f64", x0=30, y0=34, drift=v, seed=seed, stream_id=sid)

    def frame(i):
        if stall_from is not None and i >= stall_from:
            return None
        return vid.frames[i]

    return StreamRequest(sid, arrival, p, frames, fps, frame), vid


def _sched(caps, fail_on=None, stall_timeout=0.5, step_cost=0.002):
    clk = VirtualClock()
    be = FakeBackend(caps, clk, fail_on=fail_on, step_cost=step_cost)
    return Scheduler(be, clock=clk, stall_timeout=stall_timeout), clk, be


def test_every_frame_is_stepped_in_order_and_matches_the_stream_run_alone():
    s, clk, be = _sched({512: 3})
    reqs = [_stream(i, 0.05 * i) for i in range(3)]
    for r, _ in reqs:
        assert s.submit(r)
    s.run(until=100.0, sleep=clk.sleep)
    for r, vid in reqs:
        res = s.results[r.sid]
        assert res.status == "done" and res.frames_done == r.n_frames - 1
        ref = oracle.run(oracle.make_params(r.params.n_particles, SIDE, SIDE, radius=5,
                                            drift=(r.params.drift_x, r.params.drift_y),
                                            seed=0, stream_id=r.sid),
                         vid.frames, 30, 34)
        assert np.array_equal(np.array(res.estimates), ref[0][1:])


def test_admission_waits_for_a_free_slot_under_the_budget():
    s, clk, be = _sched({512: 2})
    reqs = [_stream(i, 0.0) for i in range(3)]
    for r, _ in reqs:
        s.submit(r)
    s.run(until=100.0, sleep=clk.sleep)
    st = {sid: r.status for sid, r in s.results.items()}
    assert st == {0: "done", 1: "done", 2: "done"}
    waits = sorted(r.admission_wait for r in s.results.values())
    assert waits[0] == 0.0 and waits[1] == 0.0
    # the third waits until a stream leaves: about (frames - 1) / fps
    assert waits[2] >= (6 - 1) / 10.0 - 1e-9
    assert be.high_water() == 2 * 512


def test_invalid_parameters_are_rejected_at_submission():
    s, clk, be = _sched({512: 1})
    r, _ = _stream(0, 0.0)
    r.params.disk_radius = 0
    assert not s.submit(r)
    big, _ = _stream(1, 0.0, n=4096)
    assert not s.submit(big)
    assert s.results[0].status == "rejected" and "disk_radius" in s.results[0].reason
    assert s.results[1].status == "rejected"
    assert s.idle()


def test_stalled_stream_is_evicted_and_its_slot_reused():
    s, clk, be = _sched({512: 1}, stall_timeout=0.5)
    a, _ = _stream(0, 0.0, stall_from=3)
    b, _ = _stream(1, 0.01)
    s.submit(a)
    s.submit(b)
    s.run(until=100.0, sleep=clk.sleep)
    assert s.results[0].status == "evicted" and s.results[0].frames_done == 2
    assert s.results[1].status == "done"
    # b was admitted once a's frame 3 was late by the timeout
    assert s.results[1].admission_wait >= 0.3 + 0.5 - 0.01 - 1e-9
    assert be.in_use == 0


def test_a_failed_step_fails_only_that_stream():
    s, clk, be = _sched({512: 2}, fail_on={0: 2})
    a, _ = _stream(0, 0.0)
    b, _ = _stream(1, 0.0)
    s.submit(a)
    s.submit(b)
    s.run(until=100.0, sleep=clk.sleep)
    assert s.results[0].status == "failed" and s.results[0].frames_done == 1
    assert s.results[1].status == "done" and s.results[1].frames_done == 5
    assert be.in_use == 0


def test_latency_is_frame_arrival_to_estimate_ready():
    # one stream, frames every 0.1 s, a step costs 0.01 s and the loop polls
    # every 0.001 s: each frame is picked up within a poll of its arrival
    s, clk, be = _sched({512: 1}, step_cost=0.01)
    r, _ = _stream(0, 0.0, frames=5)
    s.submit(r)
    summ = s.run(until=100.0, sleep=clk.sleep, poll=0.001)
    lat = np.array(s.latencies)
    assert lat.size == 4
    assert np.all(lat >= 0.01 - 1e-12) and np.all(lat <= 0.011 + 1e-9)
    assert summ["frames"] == 4 and summ["particle_updates"] == 4 * 300


def test_slot_plan_fits_the_budget():
    caps = slot_classes(1000, 1_000_000)
    assert caps[0] == 1024 and caps[-1] == 1 << 20
    plan = plan_pool(2 << 30, "f16", caps)
    used = sum(pf.pf_member_bytes(pf.make_params(c, 64, 64, "f16")) * k for c, k in plan.items())
    assert used <= 2 << 30 and used > 0.9 * (2 << 30)


# ---------------------------------------------------------------------------
# FrameSeq streams over a backend with the array calls: the scheduler keeps
# them in columns and steps them with no per-stream Python work; the results
# must be those of the generic path.

from paper_2308_00763_amd.serve import FrameSeq  # noqa: E402
from serve_fake import ArrayFakeBackend  # noqa: E402


def _array_sched(caps, fail_on=None, step_cost=0.002, stall_timeout=0.5):
    clk = VirtualClock()
    be = ArrayFakeBackend(caps, clk, fail_on=fail_on, step_cost=step_cost)
    return Scheduler(be, clock=clk, stall_timeout=stall_timeout), clk, be


def _seq_stream(be, sid, arrival, n=300, frames=6, fps=10.0):
    r, vid = _stream(sid, arrival, n=n, frames=frames, fps=fps)
    r.frame = be.frame_seq(sid + 1, vid.frames)
    assert isinstance(r.frame, FrameSeq)
    return r, vid


def test_column_streams_match_the_oracle_run_alone():
    s, clk, be = _array_sched({512: 3})
    reqs = [_seq_stream(be, i, 0.05 * i, frames=5 + i) for i in range(5)]
    for r, _ in reqs:
        assert s.submit(r)
    s.run(until=100.0, sleep=clk.sleep)
    assert be.array_steps > 0 and not s.due  # every stream went through the columns
    for r, vid in reqs:
        res = s.results[r.sid]
        assert res.status == "done" and res.frames_done == r.n_frames - 1
        ref = oracle.run(oracle.make_params(r.params.n_particles, SIDE, SIDE, radius=5,
                                            drift=(r.params.drift_x, r.params.drift_y),
                                            seed=0, stream_id=r.sid),
                         vid.frames, 30, 34)
        assert np.array_equal(np.array(res.estimates), ref[0][1:])
    assert be.in_use == 0


def test_column_latency_and_updates():
    s, clk, be = _array_sched({512: 1}, step_cost=0.01)
    r, _ = _seq_stream(be, 0, 0.0, frames=5)
    s.submit(r)
    summ = s.run(until=100.0, sleep=clk.sleep, poll=0.001)
    lat = np.array(s.latencies)
    assert lat.size == 4
    assert np.all(lat >= 0.01 - 1e-12) and np.all(lat <= 0.011 + 1e-9)
    assert summ["frames"] == 4 and summ["particle_updates"] == 4 * 300


def test_column_step_failure_fails_only_that_stream():
    s, clk, be = _array_sched({512: 2}, fail_on={0: 2})
    a, _ = _seq_stream(be, 0, 0.0)
    b, _ = _seq_stream(be, 1, 0.0)
    s.submit(a)
    s.submit(b)
    s.run(until=100.0, sleep=clk.sleep)
    assert s.results[0].status == "failed" and s.results[0].frames_done == 1
    assert s.results[1].status == "done" and s.results[1].frames_done == 5


def test_column_store_compaction_keeps_every_estimate():
    # many short streams through few slots: rows and estimate runs are
    # reused and the store is compacted while streams are live
    s, clk, be = _array_sched({512: 4}, step_cost=0.0005)
    s.cols.est = np.zeros((8, 2))  # a tiny store: compaction on most admissions
    reqs = [_seq_stream(be, i, 0.01 * i, n=64, frames=3 + i % 5) for i in range(24)]
    for r, _ in reqs:
        s.submit(r)
    s.run(until=1000.0, sleep=clk.sleep)
    for r, vid in reqs:
        res = s.results[r.sid]
        assert res.status == "done" and res.frames_done == r.n_frames - 1
        ref = oracle.run(oracle.make_params(64, SIDE, SIDE, radius=5, drift=(r.params.drift_x, r.params.drift_y),
                                            seed=0, stream_id=r.sid), vid.frames, 30, 34)
        assert np.array_equal(np.array(res.estimates), ref[0][1:]), r.sid
    assert not s.cols.used.any()


def test_single_frame_stream_finishes_without_a_step():
    s, clk, be = _array_sched({512: 1})
    r, _ = _seq_stream(be, 0, 0.0, frames=1)
    s.submit(r)
    s.run(until=100.0, sleep=clk.sleep)
    assert s.results[0].status == "done" and s.results[0].frames_done == 0
