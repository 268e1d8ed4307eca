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


# --------------------------------------------------------------------------
# The tuning table inside the library: PF_FLAG_TUNED filters, alone and in
# batches, run at the sizes the table gives for this GPU.

import os  # noqa: E402

from test_gpu_batch import _alone, _videos  # noqa: E402


@pytest.fixture
def arch_table():
    """This GPU's architecture name with an empty table; the shipped table is
    reinstalled after the test."""
    pf.pf_tune_clear()
    yield torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    pf.pf_tune_clear()
    if os.path.exists(pf.TUNE_TABLE):
        pf.pf_tune_load(pf.TUNE_TABLE)


def _stream_mix(ns, T, seed):
    streams = pfsynth.stream_mix(len(ns), side=128, frames=T, seed=seed)
    for s, n in zip(streams, ns):
        s.n_particles = n
    return streams


def _mk(s, dtype, **kw):
    return pf.make_params(s.n_particles, 128, 128, dtype, radius=5, x0=s.start[0], y0=s.start[1],
                          drift=s.velocity, seed=21, stream_id=s.stream_id, **kw)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
def test_tuned_batch_members_equal_their_tuned_alone_runs(arch_table, dtype):
    arch = arch_table
    # buckets: 5000 -> 13, 3000 -> 12 (nearest 13), 70001 -> 17, 300000 -> 19 (nearest 17 or 20)
    pf.pf_tune_set(arch, dtype, 13, 512, 128)
    pf.pf_tune_set(arch, dtype, 17, 128, 1024)
    pf.pf_tune_set(arch, dtype, 20, 256, 64)
    ns = [5000, 70001, 20000, 3000, 300000, 1100, 1 << 20]
    want_a = [512, 128, 256, 512, 256, 512, 256]
    tuned = [True, True, False, True, True, True, True]
    T = 5
    streams = _stream_mix(ns, T, seed=77)
    params = [_mk(s, dtype, tuned=tu) for s, tu in zip(streams, tuned)]
    vids = _videos(streams, T)
    b = pf.Batch(params)
    for k in range(len(ns)):
        ta, tc = pf.pf_launch_config(b.filter(k))
        assert ta == want_a[k], (k, ta)
        assert tc == 256  # the batch's pass C size for every member
    est_b = []
    for t in range(1, T):
        print(f"[tune] batch dtype={dtype} step={t}", flush=True)
        b.step([vids[k, t] for k in range(len(ns))])
        est_b.append(b.estimates())
    est_b = np.stack(est_b)
    for k, p in enumerate(params):
        print(f"[tune] alone dtype={dtype} filter={k} n={p.n_particles}", flush=True)
        est_a, got_a = _alone(p, vids[k], range(1, T))
        assert np.array_equal(est_a, est_b[:, k, :]), k
        got_b = b.export(k)
        assert np.array_equal(got_a["x"], got_b["x"]) and np.array_equal(got_a["y"], got_b["y"]), k
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_tuned_filter_equals_the_same_sizes_given_explicitly(arch_table, dtype):
    arch = arch_table
    pf.pf_tune_set(arch, dtype, 17, 512, 1024)
    T = 6
    (s,) = _stream_mix([70001], T, seed=5)
    vids = _videos([s], T)
    f = pf.Filter(_mk(s, dtype, tuned=True))
    assert f.launch_config() == (512, 1024)
    f.close()
    est_t, got_t = _alone(_mk(s, dtype, tuned=True), vids[0], range(1, T))
    est_e, got_e = _alone(_mk(s, dtype, threads_a=512, threads_c=1024), vids[0], range(1, T))
    assert np.array_equal(est_t, est_e)
    assert np.array_equal(got_t["x"], got_e["x"]) and np.array_equal(got_t["y"], got_e["y"])
    # an untuned filter keeps the defaults whatever the table holds
    g = pf.Filter(_mk(s, dtype))
    assert g.launch_config() == (256, 256)
    g.close()


def test_reinit_moves_a_member_to_its_new_tuned_size(arch_table):
    arch = arch_table
    pf.pf_tune_set(arch, "f16", 12, 512, 0)
    pf.pf_tune_set(arch, "f16", 18, 128, 0)
    T = 6
    streams = _stream_mix([4000, 200000, 9000], T, seed=9)
    vids = _videos(streams, T)
    params = [_mk(s, "f16", tuned=True) for s in streams]
    b = pf.Batch(params)
    assert [pf.pf_launch_config(b.filter(k))[0] for k in range(3)] == [512, 128, 512]
    for t in range(1, 3):
        b.step([vids[k, t] for k in range(3)])
    # filter 1 restarts with 4000 particles (bucket 12): pass A at 512 threads
    streams[1].n_particles = 4000
    p1 = _mk(streams[1], "f16", tuned=True)
    b.reinit(1, p1)
    assert pf.pf_launch_config(b.filter(1))[0] == 512
    for t in range(1, 4):
        b.step([vids[k, t] for k in range(3)], np.array([0, 1, 0], np.uint8))
    est_a, got_a = _alone(p1, vids[1], range(1, 4))
    got_b = b.export(1)
    assert np.array_equal(got_a["x"], got_b["x"]) and np.array_equal(got_a["y"], got_b["y"])
    assert np.array_equal(est_a[-1], b.estimates()[1])
    b.close()


def test_replayed_graph_of_a_batch_with_mixed_pass_a_sizes(arch_table):
    arch = arch_table
    pf.pf_tune_set(arch, "f16", 13, 512, 0)
    pf.pf_tune_set(arch, "f16", 17, 128, 0)
    T = 5
    ns = [5000, 70001, 20000, 1 << 20, 6000]
    streams = _stream_mix(ns, T, seed=31)
    params = [_mk(s, "f16", tuned=k != 2) for k, s in enumerate(streams)]
    vids = _videos(streams, T)
    ref = pf.Batch(params)
    for t in range(1, T):
        ref.step([vids[k, t] for k in range(len(ns))])
    e_est = ref.estimates()
    e_got = [ref.export(k) for k in range(len(ns))]
    ref.close()
    side = torch.cuda.Stream()
    b = pf.Batch(params, stream=side)
    static = torch.zeros_like(vids[:, 0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.step([static[k] for k in range(len(ns))])
    torch.cuda.synchronize()
    for t in range(1, T):
        print(f"[tune] graph replay {t}", flush=True)
        static.copy_(vids[:, t])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
    assert np.array_equal(b.estimates(), e_est)
    for k in range(len(ns)):
        got = b.export(k)
        assert np.array_equal(got["x"], e_got[k]["x"]) and np.array_equal(got["y"], e_got[k]["y"]), k
    b.close()


def test_shipped_table_resolves_for_this_gpu():
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    rows = [ln.split("#", 1)[0].split() for ln in open(pf.TUNE_TABLE)]
    rows = [r for r in rows if r and r[0] == arch]
    assert rows, f"the shipped table has no entry for {arch}"
    for _, dt, bkt, ta, tc in rows:
        n = 1 << int(bkt)
        if n > (1 << 22):
            continue
        f = pf.Filter(pf.make_params(n, 256, 256, dt, tuned=True, x0=128, y0=128))
        got = f.launch_config()
        f.close()
        assert got[0] == (int(ta) or 256), (dt, bkt, got)
        if int(tc):
            assert got[1] == int(tc), (dt, bkt, got)
