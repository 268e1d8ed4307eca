"""GPU tests of the deferred resampling of single filters: an FP64 or FP32
filter of at most 2^20 particles resampling systematically skips pass C and
the next step's pass A gathers the resampled particles for its tiles (the
16-bit modes resample at once and must give the same results as well).  Every step must give
the results of resampling at once (a batch member, which always runs pass C)
bit for bit: estimates after every step, the state exported mid-run (which
runs the pending resampling) and at the end, the propagated positions of odd
and even steps (the two sets of step outputs), graph replays, and a resume
from an exported checkpoint."""
import numpy as np
import pytest
import torch

import paper_2308_00763_amd as pf
import pfsynth

pytestmark = pytest.mark.gpu

SIDE = 128


def _stream(n, T, seed):
    s = pfsynth.stream_mix(1, side=SIDE, frames=T, seed=seed)[0]
    s.n_particles = n
    vid = torch.from_numpy(pfsynth.stream_video(s, SIDE, T).frames).to("cuda:0")
    p = pf.make_params(n, SIDE, SIDE, "f16", x0=s.start[0], y0=s.start[1], drift=s.velocity, seed=11,
                       stream_id=s.stream_id)
    return s, vid, p


def _params(s, n, dtype):
    return pf.make_params(n, SIDE, SIDE, dtype, x0=s.start[0], y0=s.start[1], drift=s.velocity, seed=11,
                          stream_id=s.stream_id)


def _same_state(a, b):
    return a["t"] == b["t"] and np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("n", [1, 1000, 1023, 5000, 70001, 300001, 1 << 20])
def test_deferred_resampling_equals_resampling_at_once(dtype, n):
    T = 10
    s, vid, _ = _stream(n, T, seed=300 + n % 97)
    p = _params(s, n, dtype)
    alone = pf.Filter(p)
    b = pf.Batch([p])
    member = b.filter(0)
    for t in range(1, T):
        print(f"[deferred] dtype={dtype} n={n} step={t}", flush=True)
        alone.step(vid[t])
        b.step([vid[t]])
        assert np.array_equal(np.array(alone.estimate()), b.estimates()[0]), t
        if t in (3, 4):  # the outputs of an odd and of an even step
            ga = pf.pf_export_step(alone.handle, n)
            gb = pf.pf_export_step(member, n)
            assert np.array_equal(ga["x_prop"], gb["x_prop"]) and np.array_equal(ga["y_prop"], gb["y_prop"]), t
        if t in (5, 6):  # runs the pending resampling; the next step reads the state
            assert _same_state(alone.export(), b.export(0)), t
    assert _same_state(alone.export(), b.export(0))
    alone.close()
    b.close()


def test_deferred_filters_run_no_pass_c():
    # a deferring filter leaves its resampling pending after each step (the
    # device block's flag, the word after the step count) and runs no pass C;
    # an export runs the pending resampling and clears the flag; a filter with
    # diagnostics, with an explicit pass-C size or in a 16-bit mode resamples
    # at once
    T = 6
    s, vid, _ = _stream(1 << 20, T, seed=17)
    res = {}
    for dt, diag, tc in (("f32", False, None), ("f32", True, None), ("f64", False, 256), ("f16", False, None)):
        p = pf.make_params(1 << 20, SIDE, SIDE, dt, x0=s.start[0], y0=s.start[1], drift=s.velocity, seed=11,
                           diagnostics=diag, threads_c=tc)
        f = pf.Filter(p)
        pend = lambda: int(f.workspace[4:8].view(torch.int32).item())  # noqa: E731
        assert pend() == 0
        f.step(vid[1])
        pf.pf_profile_start(f.handle, 4)
        for t in range(2, T):
            f.step(vid[t])
        res[(dt, diag)] = pf.pf_profile_read(f.handle)
        torch.cuda.synchronize()
        defers = not diag and tc is None and dt in ("f32", "f64")
        assert pend() == (1 if defers else 0)
        f.export()
        assert pend() == 0
        f.close()
    a_ms, _, c_ms, steps = res[("f32", False)]
    assert steps == 4 and a_ms > 0 and c_ms == 0.0, res
    assert res[("f32", True)][2] > 0.0 and res[("f64", False)][2] > 0.0 and res[("f16", False)][2] > 0.0, res


@pytest.mark.parametrize("dtype,n", [("f32", 70001), ("f32", 1 << 20), ("f64", 3000)])
def test_deferred_graph_replays_equal_eager_steps(dtype, n):
    # one captured step replayed; eager steps of a reference filter between
    # the replays; an export after the third replay runs the pending
    # resampling between two replays
    T = 9
    s, vid, _ = _stream(n, T, seed=41)
    p = _params(s, n, dtype)
    eager = pf.Filter(p)
    side = torch.cuda.Stream()
    f = pf.Filter(p, stream=side)
    static = torch.zeros((SIDE, SIDE), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        pf.pf_step(f.handle, static.data_ptr(), SIDE)
    torch.cuda.synchronize()
    for t in range(1, T):
        print(f"[deferred-graph] dtype={dtype} n={n} replay={t}", flush=True)
        eager.step(vid[t])
        static.copy_(vid[t])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(np.array(f.estimate()), np.array(eager.estimate())), t
        if t == 3:
            assert _same_state(f.export(), eager.export())
    assert _same_state(f.export(), eager.export())
    f.close()
    eager.close()


def test_resume_from_a_checkpoint_of_a_deferring_filter():
    # FP64: an imported state is the exported one exactly (the reduced modes
    # store offsets from an origin that an import chooses afresh)
    T = 10
    s, vid, _ = _stream(5000, T, seed=77)
    p = _params(s, 5000, "f64")
    ref = pf.Filter(p)
    for t in range(1, T):
        ref.step(vid[t])
    want = ref.export()
    ref.close()
    a = pf.Filter(p)
    for t in range(1, 5):
        a.step(vid[t])
    ck = a.export()
    a.close()
    b = pf.Filter(p)
    b.load(ck["x"], ck["y"], ck["t"])
    for t in range(5, T):
        b.step(vid[t])
    assert _same_state(b.export(), want)
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_import_over_a_pending_resampling(dtype):
    # an import into a filter whose last resampling is pending replaces the
    # state: the next steps equal those of a fresh filter given the same state
    T = 8
    n = 5000
    s, vid, _ = _stream(n, T, seed=91)
    p = _params(s, n, dtype)
    rng = np.random.default_rng(5)
    x = s.start[0] + rng.normal(0, 2, n)
    y = s.start[1] + rng.normal(0, 2, n)
    a = pf.Filter(p)
    for t in range(1, 4):
        a.step(vid[t])
    a.load(x, y, 3)
    b = pf.Filter(p)
    b.load(x, y, 3)
    for t in range(4, T):
        a.step(vid[t])
        b.step(vid[t])
        assert np.array_equal(np.array(a.estimate()), np.array(b.estimate())), t
    assert _same_state(a.export(), b.export())
    a.close()
    b.close()
