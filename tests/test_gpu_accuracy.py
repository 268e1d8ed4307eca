"""The paper's accuracy experiment (Sec. 5, verification paragraph): a
512x512, 100-frame video of a disk moving toward y = 0 and bouncing off it,
tracked with 128 particles in every precision.  The double filter follows the
ground truth; the single-precision predictions match the double ones; the
16-bit modes stay comparable.  The GPU's FP64 track is also checked against the
oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2308_00763_amd as pf
import pfsynth

pytestmark = pytest.mark.gpu


def _track(dtype, w, frames_dev, centres):
    p = pf.make_params(w.n_particles, w.width, w.height, dtype, radius=w.radius,
                       x0=centres[0][0], y0=centres[0][1], drift=w.drift, sigma=w.sigma,
                       seed=w.filter_seed)
    f = pf.Filter(p)
    est = [tuple(centres[0])]
    for t in range(1, frames_dev.shape[0]):
        f.step(frames_dev[t])
        est.append(f.estimate())
    f.close()
    return np.array(est)


def test_bounce_accuracy_in_every_precision():
    w = pfsynth.WORKLOADS["bounce512_n128"]
    vid = pfsynth.workload_video(w, bounce=True)
    fr = torch.from_numpy(vid.frames).to("cuda:0")
    op = oracle.make_params(w.n_particles, w.width, w.height, radius=w.radius, drift=w.drift,
                            sigma=w.sigma, seed=w.filter_seed)
    ref, _, _ = oracle.run(op, vid.frames, *vid.centres[0])
    tr = {dt: _track(dt, w, fr, vid.centres) for dt in ("f64", "f32", "f16", "bf16")}
    rms = {dt: float(np.sqrt(np.mean(np.sum((e - vid.centres) ** 2, axis=1)))) for dt, e in tr.items()}
    dev = {dt: float(np.max(np.hypot(*(e - tr["f64"]).T))) for dt, e in tr.items()}
    print(f"[accuracy] RMS vs truth {rms}; max deviation from FP64 {dev}; "
          f"oracle RMS {np.sqrt(np.mean(np.sum((ref - vid.centres) ** 2, axis=1))):.4f}", flush=True)
    assert np.max(np.abs(tr["f64"] - ref)) <= 1e-6
    assert rms["f64"] <= 2.0
    assert dev["f32"] <= 1e-3
    for dt in ("f16", "bf16"):
        assert rms[dt] <= rms["f64"] + 1.0
