"""Pins of the oracle's weighting, normalising, estimate and systematic
resampling (paper Sec. 4, Eq. (5), normalizing and resampling paragraphs).

Pins from outside the oracle:
  * scipy.special.softmax of the log-likelihoods gives the normalised weights;
  * exact rational brute force at N <= 8 (fractions.Fraction): the ancestors of
    systematic resampling, the offspring counts floor(N w) / ceil(N w), and the
    expectation over u0 of every count, N w_i, found by enumerating the u0
    breakpoints;
  * special cases: uniform weights, the u0 = 0 tie, one-hot weights, N = 1;
  * invariants: sum w = 1, C monotone with C_{N-1} = 1, the estimate is the
    weighted mean before resampling.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import softmax

import oracle


def _exact_ancestors(w_float, u0):
    """Systematic resampling in exact rationals on the exact float weights."""
    n = len(w_float)
    w = [Fraction(float(v)) for v in w_float]
    tot = sum(w)
    C = []
    acc = Fraction(0)
    for v in w:
        acc += v
        C.append(acc / tot)
    u0 = Fraction(float(u0))
    anc = []
    for j in range(n):
        uj = (j + u0) / n
        a = next((i for i in range(n) if C[i] >= uj), n - 1)
        anc.append(a)
    return anc, C


def _min_gap(C, u0, n):
    gaps = [abs(float(c) - (j + u0) / n) for c in C for j in range(n)]
    return min(gaps)


def _rand_case(rng, n):
    L = rng.normal(0, 2.0, n)
    x = rng.normal(0, 10, n)
    y = rng.normal(0, 10, n)
    return L, x, y


def test_weights_are_softmax_and_cdf_invariants():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 100, 4096):
        L, x, y = _rand_case(rng, n)
        L = L * 30  # wide range of log-weights
        out = oracle.reweight_resample(L, x, y, 0.37)
        np.testing.assert_allclose(out["w"], softmax(L), rtol=1e-12, atol=1e-300)
        assert abs(out["w"].sum() - 1.0) < 1e-12
        assert np.all(np.diff(out["cdf"]) >= 0)
        assert out["cdf"][-1] == 1.0
        # estimate = weighted mean before resampling
        assert out["est"][0] == pytest.approx(float(np.dot(softmax(L), x)), rel=1e-12, abs=1e-12)
        assert out["est"][1] == pytest.approx(float(np.dot(softmax(L), y)), rel=1e-12, abs=1e-12)
        # commit: positions are copies of the ancestors
        np.testing.assert_array_equal(out["x"], x[out["anc"]])
        np.testing.assert_array_equal(out["y"], y[out["anc"]])
        assert np.all(np.diff(out["anc"]) >= 0)


def test_previous_weights_enter_eq5():
    rng = np.random.default_rng(1)
    L, x, y = _rand_case(rng, 16)
    wp = rng.uniform(0.1, 1.0, 16)
    out = oracle.reweight_resample(L, x, y, 0.5, w_prev=wp)
    want = wp * np.exp(L - L.max())
    np.testing.assert_allclose(out["w"], want / want.sum(), rtol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_bruteforce_ancestors(n):
    rng = np.random.default_rng(100 + n)
    checked = 0
    for trial in range(200):
        L, x, y = _rand_case(rng, n)
        u0 = rng.uniform()
        out = oracle.reweight_resample(L, x, y, u0)
        anc, C = _exact_ancestors(out["w"], u0)
        if _min_gap(C, u0, n) < 1e-12:
            continue  # a tie at float resolution: either side is correct
        assert list(out["anc"]) == anc
        checked += 1
    assert checked > 150


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_bruteforce_offspring_counts_and_expectation(n):
    rng = np.random.default_rng(7 + n)
    for trial in range(20):
        L, x, y = _rand_case(rng, n)
        out0 = oracle.reweight_resample(L, x, y, 0.5)
        w = out0["w"]
        wf = [Fraction(float(v)) for v in w]
        tot = sum(wf)
        Cx = np.cumsum([float(v / tot) for v in wf])
        # u0 breakpoints: counts change where (j + u0) / n crosses some C_i
        bps = sorted(set([0.0, 1.0] + [float((n * c) % 1.0) for c in Cx]))
        expect = np.zeros(n)
        for a, b in zip(bps[:-1], bps[1:]):
            if b - a < 1e-9:
                continue
            mid = 0.5 * (a + b)
            out = oracle.reweight_resample(L, x, y, mid)
            counts = np.bincount(out["anc"], minlength=n)
            assert counts.sum() == n
            nw = n * w
            assert np.all((counts == np.floor(nw)) | (counts == np.ceil(nw)))
            expect += (b - a) * counts
        np.testing.assert_allclose(expect, n * w, atol=1e-7)


def test_uniform_weights_and_u0_tie():
    n = 64
    L = np.zeros(n)
    x = np.arange(n, dtype=float)
    out = oracle.reweight_resample(L, x, x, 0.3)
    assert np.all(out["w"] == 1.0 / n)
    assert list(out["anc"]) == list(range(n))
    # u0 = 0: u_j = j / n coincides with C_{j-1} = j / n, and ">=" picks j - 1
    out = oracle.reweight_resample(L, x, x, 0.0)
    assert list(out["anc"]) == [0] + list(range(n - 1))


def test_one_hot_and_single_particle():
    n = 50
    L = np.full(n, -1e4)
    L[17] = 0.0
    x = np.arange(n, dtype=float)
    out = oracle.reweight_resample(L, x, x, 0.99)
    assert np.all(out["anc"] == 17)
    assert out["est"][0] == 17.0
    out = oracle.reweight_resample(np.array([3.0]), np.array([1.5]), np.array([2.5]), 0.4)
    assert list(out["anc"]) == [0] and out["w"][0] == 1.0
    assert list(out["est"]) == [1.5, 2.5]
