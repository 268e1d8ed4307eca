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


def _fleet(n_filters, dtype, T, side=128, seed=51):
    streams = pfsynth.stream_mix(n_filters, side=side, frames=T, seed=seed, n_lo=300, n_hi=300000)
    streams[0].n_particles = 1_500_000   # a filter of more than 1024 tiles
    streams[4].n_particles = 4_300_000   # and one of more than 4096 (grouped combine)
    params = [pf.make_params(s.n_particles, side, side, dtype, radius=5, x0=s.start[0], y0=s.start[1],
                             drift=s.velocity, seed=4, stream_id=s.stream_id) for s in streams]
    vids = torch.from_numpy(np.stack([pfsynth.stream_video(s, side, T).frames for s in streams])).to("cuda:0")
    return params, vids


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_replayed_batch_graph_equals_eager_batch(dtype):
    # filters of every combine class; the graph steps a
    # fixed active subset; eager steps of the other filters run between the
    # replays (they rewrite the device plan, which each replay uploads again)
    T, nf = 6, 9
    params, vids = _fleet(nf, dtype, T)
    active = np.array([1, 1, 0, 1, 1, 1, 0, 1, 1], np.uint8)
    rest = (1 - active).astype(np.uint8)

    ref = pf.Batch(params)
    for t in range(1, T):
        ref.step([vids[k, t] for k in range(nf)], active)
        ref.step([vids[k, t] for k in range(nf)], rest)
    e_est = ref.estimates()
    e_got = [ref.export(k) for k in range(nf)]
    ref.close()

    side = torch.cuda.Stream()
    b = pf.Batch(params, stream=side)
    static = torch.zeros_like(vids[:, 0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.step([static[k] for k in range(nf)], active)
    torch.cuda.synchronize()
    assert [b.export(k)["t"] for k in range(nf)] == [0] * nf  # recorded, not run
    for t in range(1, T):
        print(f"[graph] batch {dtype} replay {t}", flush=True)
        static.copy_(vids[:, t])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.step([vids[k, t] for k in range(nf)], rest)
        torch.cuda.synchronize()
    g_est = b.estimates()
    assert np.array_equal(g_est, e_est)
    for k in range(nf):
        got = b.export(k)
        assert got["t"] == e_got[k]["t"] == T - 1
        assert np.array_equal(got["x"], e_got[k]["x"]) and np.array_equal(got["y"], e_got[k]["y"]), k
    b.close()
