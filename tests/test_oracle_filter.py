"""End-to-end pins of the oracle's SIR filter.

  * Kalman filter: with the disk likelihood swapped for a Gaussian observation
    of the position, the model is linear-Gaussian and the scalar Kalman filter
    per axis gives the exact posterior mean.  The oracle's propagation, weights,
    estimate and resampling (everything but the disk likelihood) must converge
    to it as N grows, within a Monte Carlo envelope c * sqrt(P / N).
  * Propagation with sigma = 0 moves every particle by exactly t * d.
  * On the 128x128, 10-frame, N = 1000 moving-disk video the FP64 track stays
    within 1 px of the ground truth on every frame (paper Sec. 5: the double
    version follows the ground truth).
"""
import numpy as np
import pytest

import oracle
import pfsynth


def _kalman_run(n, steps, seed, R=4.0, d=(1.0, -2.0), sig=(5.0, 2.0)):
    rng = np.random.default_rng(seed)
    truth = np.zeros(2)
    p = oracle.make_params(n, 64, 64, drift=d, sigma=sig, seed=seed, stream_id=3)
    x = np.zeros(n)
    y = np.zeros(n)
    m = np.zeros(2)
    P = np.zeros(2)
    errs = []
    envs = []
    for t in range(1, steps + 1):
        truth = truth + np.array(d) + np.array(sig) * rng.standard_normal(2)
        obs = truth + np.sqrt(R) * rng.standard_normal(2)
        # Kalman predict / update per axis
        mp = m + np.array(d)
        Pp = P + np.array(sig) ** 2
        K = Pp / (Pp + R)
        m = mp + K * (obs - mp)
        P = (1 - K) * Pp
        # particle filter step with the oracle (Gaussian observation model)
        xp, yp = oracle.propagate(p, t, x, y)
        L = -((xp - obs[0]) ** 2 + (yp - obs[1]) ** 2) / (2 * R)
        out = oracle.reweight_resample(L, xp, yp, oracle.u0(p.seed, p.stream_id, t))
        x, y = out["x"], out["y"]
        errs.append(np.abs(out["est"] - m))
        envs.append(np.sqrt(Pp / n))
    return np.array(errs), np.array(envs)


def test_kalman_convergence():
    worst = {}
    for n in (1000, 10_000, 100_000):
        errs, envs = _kalman_run(n, steps=8, seed=11)
        assert np.all(errs <= 6.0 * envs), (n, errs / envs)
        worst[n] = errs.max()
    # the error shrinks roughly like 1/sqrt(N): at least 3x over two decades
    assert worst[100_000] < worst[1000] / 3.0


def test_kalman_detects_a_wrong_drift():
    # The same check fails when the propagation uses the wrong drift sign
    # (the Eq. (2) sign reading): guards the power of the envelope test.
    n = 20_000
    rng = np.random.default_rng(5)
    d, sig, R = np.array([1.0, -2.0]), np.array([5.0, 2.0]), 4.0
    p = oracle.make_params(n, 64, 64, drift=(1.0, 2.0), sigma=(5.0, 2.0), seed=1)
    x = np.zeros(n); y = np.zeros(n)
    truth = np.zeros(2); m = np.zeros(2); P = np.zeros(2)
    bad = 0
    for t in range(1, 7):
        truth = truth + d + sig * rng.standard_normal(2)
        obs = truth + np.sqrt(R) * rng.standard_normal(2)
        mp = m + d; Pp = P + sig ** 2; K = Pp / (Pp + R)
        m = mp + K * (obs - mp); P = (1 - K) * Pp
        xp, yp = oracle.propagate(p, t, x, y)
        L = -((xp - obs[0]) ** 2 + (yp - obs[1]) ** 2) / (2 * R)
        out = oracle.reweight_resample(L, xp, yp, oracle.u0(p.seed, p.stream_id, t))
        x, y = out["x"], out["y"]
        bad += int(np.abs(out["est"][1] - m[1]) > 6.0 * np.sqrt(Pp[1] / n))
    assert bad >= 3


def test_zero_noise_moves_by_drift():
    n = 33
    p = oracle.make_params(n, 64, 64, drift=(1.0, -2.0), sigma=(0.0, 0.0))
    x = np.full(n, 10.25)
    y = np.full(n, 40.5)
    for t in range(1, 6):
        x, y = oracle.propagate(p, t, x, y)
    assert np.all(x == 15.25) and np.all(y == 30.5)


def test_propagation_increment_distribution():
    n = 200_000
    p = oracle.make_params(n, 64, 64, drift=(1.0, -2.0), sigma=(5.0, 2.0), seed=9)
    x0 = np.random.default_rng(0).uniform(0, 100, n)
    y0 = np.random.default_rng(1).uniform(0, 100, n)
    x, y = oracle.propagate(p, 4, x0, y0)
    dx, dy = x - x0, y - y0
    assert abs(dx.mean() - 1.0) < 5 * 5 / np.sqrt(n)
    assert abs(dy.mean() + 2.0) < 5 * 2 / np.sqrt(n)
    assert abs(dx.std() - 5.0) < 0.05 and abs(dy.std() - 2.0) < 0.02


def test_tracks_the_disk_within_one_pixel():
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w)
    p = oracle.make_params(w.n_particles, w.width, w.height, radius=w.radius,
                           drift=w.drift, sigma=w.sigma, seed=w.filter_seed)
    est, x, y = oracle.run(p, vid.frames, *vid.centres[0])
    err = np.linalg.norm(est - vid.centres, axis=1)
    assert np.all(err <= 1.0), err


def test_step_is_the_composition_of_its_parts():
    w = pfsynth.WORKLOADS["disk128_n1000"]
    vid = pfsynth.workload_video(w, frames=3)
    n = 257
    p = oracle.make_params(n, w.width, w.height, radius=w.radius, seed=4, stream_id=2)
    x = np.full(n, 64.0)
    y = np.full(n, 64.0)
    s = oracle.step(p, 1, vid.frames[1], x, y)
    xp, yp = oracle.propagate(p, 1, x, y)
    np.testing.assert_array_equal(s["x_prop"], xp)
    L = oracle.likelihood(p, vid.frames[1], xp, yp)
    np.testing.assert_array_equal(s["L"], L)
    r = oracle.reweight_resample(L, xp, yp, oracle.u0(4, 2, 1))
    np.testing.assert_array_equal(s["anc"], r["anc"])
    np.testing.assert_array_equal(s["x"], r["x"])
    np.testing.assert_array_equal(s["est"], r["est"])
