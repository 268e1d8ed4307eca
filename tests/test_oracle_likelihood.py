"""Pins of the oracle's pixel set and likelihood (paper Sec. 4, Eq. (3)-(4)).

Pins that do not come from the oracle itself:
  * the disk sizes 69 (r = 5) and 193 (r = 8), fixed by the workloads' "about 69
    offsets", and its 4-fold symmetry;
  * a closed form: each per-pixel term (I - bg)^2 - (I - fg)^2 equals
    2 (fg - bg) I - (fg^2 - bg^2), so with MEAN normalisation
    L = (2 (fg - bg) mean(I) - (fg^2 - bg^2)) / kappa, i.e.
    L = 5.12 mean(I) - 839.68 for (fg, bg, kappa) = (228, 100, 50);
    mean(I) is taken here with numpy over an edge-padded frame and a mask;
  * special cases: an all-foreground disk gives +327.68, all-background -327.68;
  * translation invariance and the half-up pixel rounding.
"""
import numpy as np
import pytest

import oracle


def test_disk_sizes_and_symmetry():
    for r, n in ((5, 69), (8, 193), (1, 1), (2, 9), (3, 25)):
        dx, dy = oracle.disk(r)
        assert dx.size == n, r
        pts = set(zip(dx.tolist(), dy.tolist()))
        for (a, b) in list(pts):
            assert (-a, b) in pts and (a, -b) in pts and (b, a) in pts
            assert a * a + b * b < r * r
        # strict: points on the circle are excluded
        assert (r, 0) not in pts and (0, r) not in pts
        # row-major order (dy, then dx)
        order = list(zip(dy.tolist(), dx.tolist()))
        assert order == sorted(order)


def _mean_over_disk(frame, cx, cy, r):
    """Mean intensity over the strict disk, outside pixels taken from an
    edge-replicated (np.pad mode="edge") frame."""
    pad = 64
    F = np.pad(frame.astype(np.float64), pad, mode="edge")
    ys, xs = np.mgrid[-r:r + 1, -r:r + 1]
    mask = xs ** 2 + ys ** 2 < r * r
    win = F[cy - r + pad: cy + r + 1 + pad, cx - r + pad: cx + r + 1 + pad]
    return win[mask].mean()


@pytest.mark.parametrize("r", [5, 8])
def test_likelihood_closed_form(r):
    rng = np.random.default_rng(11)
    H, W = 40, 56
    frame = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    p = oracle.make_params(1, W, H, radius=r)
    xs = rng.uniform(-3, W + 2, 400)
    ys = rng.uniform(-3, H + 2, 400)
    L = oracle.likelihood(p, frame, xs, ys)
    for k in range(xs.size):
        cx, cy = int(np.floor(xs[k] + 0.5)), int(np.floor(ys[k] + 0.5))
        m = _mean_over_disk(frame, cx, cy, r)
        want = 5.12 * m - 839.68
        assert L[k] == pytest.approx(want, rel=1e-12, abs=1e-10)


def test_likelihood_sum_normalisation_and_other_intensities():
    rng = np.random.default_rng(5)
    frame = rng.integers(0, 256, size=(30, 30), dtype=np.uint8)
    r, fg, bg, kappa = 5, 200, 30, 20.0
    pm = oracle.make_params(1, 30, 30, radius=r, fg=fg, bg=bg, kappa=kappa, lik_norm=oracle.MEAN)
    ps = oracle.make_params(1, 30, 30, radius=r, fg=fg, bg=bg, kappa=kappa, lik_norm=oracle.SUM)
    x, y = np.array([12.2]), np.array([14.7])
    m = _mean_over_disk(frame, 12, 15, r)
    want_mean = (2 * (fg - bg) * m - (fg * fg - bg * bg)) / kappa
    assert oracle.likelihood(pm, frame, x, y)[0] == pytest.approx(want_mean, rel=1e-12)
    assert oracle.likelihood(ps, frame, x, y)[0] == pytest.approx(want_mean * 69, rel=1e-12)


def test_all_foreground_and_background():
    p = oracle.make_params(1, 32, 32)
    fgf = np.full((32, 32), 228, np.uint8)
    bgf = np.full((32, 32), 100, np.uint8)
    assert oracle.likelihood(p, fgf, [10.0], [10.0])[0] == pytest.approx(327.68, abs=1e-12)
    assert oracle.likelihood(p, bgf, [10.0], [10.0])[0] == pytest.approx(-327.68, abs=1e-12)


def test_translation_invariance():
    rng = np.random.default_rng(2)
    frame = rng.integers(0, 256, size=(64, 64), dtype=np.uint8)
    shifted = np.zeros_like(frame)
    shifted[3:, 5:] = frame[:-3, :-5]
    p = oracle.make_params(1, 64, 64)
    for (x, y) in [(20.3, 20.6), (30.0, 41.49), (40.51, 25.2)]:
        a = oracle.likelihood(p, frame, [x], [y])[0]
        b = oracle.likelihood(p, shifted, [x + 5], [y + 3])[0]
        assert a == b


def test_half_up_rounding_of_the_particle_pixel():
    # a frame whose columns are distinguishable: L depends on the chosen column
    frame = np.tile(np.arange(64, dtype=np.uint8) * 3, (64, 1))
    p = oracle.make_params(1, 64, 64)
    L = lambda x: oracle.likelihood(p, frame, [x], [30.0])[0]
    assert L(20.5) == L(21.0) == L(21.49999)
    assert L(20.49999) == L(20.0) != L(20.5)
    # negative coordinates: floor(-0.5 + 0.5) = 0, floor(-0.51 + 0.5) = -1
    assert L(-0.5) == L(0.0)
    assert L(-0.51) == L(-1.0)


def test_edge_clamping_equals_edge_padding():
    rng = np.random.default_rng(9)
    frame = rng.integers(0, 256, size=(20, 24), dtype=np.uint8)
    p = oracle.make_params(1, 24, 20, radius=5)
    for (cx, cy) in [(0, 0), (23, 19), (-4, 7), (30, 30), (12, -6)]:
        m = _mean_over_disk(frame, cx, cy, 5)
        assert oracle.likelihood(p, frame, [float(cx)], [float(cy)])[0] == pytest.approx(
            5.12 * m - 839.68, rel=1e-12, abs=1e-10)
