"""Pins of the oracle's rejection resampler (Murray, Lee & Jacob 2016) by the
distribution it must produce, not by its formula.  Slot j proposes its own
particle first and accepts a proposal c with probability r_c = w_c / w_max,
else proposes a uniform particle, so

    P(a_j = i) = [i = j] r_j + (1 - r_j) w_i / W,        W = sum(w),
    E[offspring of i] = N w_i / W                          (unbiased),
    E[trials of slot j] = 1 + (1 - r_j) N w_max / W.

A wrong starting proposal, a wrong acceptance ratio (e.g. against the mean
instead of the maximum) or a proposal that is not uniform breaks one of the
tests below."""
import numpy as np
from scipy import stats

import oracle

W8 = np.arange(1, 9, dtype=float)  # weights 1..8 of eight particles


def _draws(L, steps, cap=4096, seed=3, sid=2):
    anc, trials = [], []
    for t in range(1, steps + 1):
        a, _, tr = oracle.rejection(L, cap, seed, sid, t)
        anc.append(a)
        trials.append(tr)
    return np.array(anc), np.array(trials)


def test_each_slot_follows_its_closed_form_distribution():
    L = np.log(W8)
    anc, _ = _draws(L, 6000)
    r = W8 / W8.max()
    for j in range(8):
        counts = np.bincount(anc[:, j], minlength=8)
        if r[j] == 1.0:   # the heaviest particle accepts its own proposal
            assert counts[j] == anc.shape[0]
            continue
        expected = (1 - r[j]) * W8 / W8.sum()
        expected[j] += r[j]
        assert stats.chisquare(counts, expected * anc.shape[0]).pvalue > 1e-4, j


def test_offspring_counts_are_unbiased():
    # E[count_i] = N w_i / W exactly; 6000 steps, 5 sigma per particle
    L = np.log(W8)
    anc, _ = _draws(L, 6000)
    counts = np.stack([np.bincount(a, minlength=8) for a in anc])
    mean = counts.mean(axis=0)
    target = 8 * W8 / W8.sum()
    se = counts.std(axis=0, ddof=1) / np.sqrt(counts.shape[0])
    assert np.all(np.abs(mean - target) < 5 * se + 1e-12), (mean, target)
    assert np.all(counts.sum(axis=1) == 8)


def test_mean_trials_match_the_acceptance_probability():
    L = np.log(W8)
    _, trials = _draws(L, 6000)
    r = W8 / W8.max()
    expected = 1 + (1 - r) * 8 * W8.max() / W8.sum()
    mean = trials.mean(axis=0)
    se = trials.std(axis=0, ddof=1) / np.sqrt(trials.shape[0])
    assert np.all(np.abs(mean - expected) < 5 * se + 1e-12), (mean, expected)


def test_uniform_weights_keep_every_slot_in_one_trial():
    n = 10_000
    anc, margin, trials = oracle.rejection(np.zeros(n), 4096, 5, 1, 3)
    assert np.array_equal(anc, np.arange(n))
    assert np.all(trials == 1)


def test_the_maximum_is_always_accepted_and_a_dominant_particle_takes_every_slot():
    n, h = 64, 17
    L = np.full(n, -1000.0)
    L[h] = 0.0
    anc, _, trials = oracle.rejection(L, 4096, 9, 4, 1)
    assert np.all(anc == h)
    assert trials[h] == 1
    # proposals are uniform: the trials until h is proposed are geometric with
    # p = 1/n after the first (rejected) own proposal, mean 1 + n
    _, tr = _draws(L, 300, seed=9, sid=4)
    rest = np.delete(tr, h, axis=1).ravel()
    se = rest.std(ddof=1) / np.sqrt(rest.size)
    assert abs(rest.mean() - (1 + n)) < 5 * se


def test_a_common_shift_changes_no_decision():
    rng = np.random.default_rng(2)
    L = rng.normal(scale=3.0, size=5000)
    a0, m0, t0 = oracle.rejection(L, 4096, 1, 7, 2)
    a1, m1, t1 = oracle.rejection(L + 17.25, 4096, 1, 7, 2)
    sure = (m0 > 1e-9) & (m1 > 1e-9)
    assert sure.mean() > 0.99
    assert np.array_equal(a0[sure], a1[sure])
    assert np.array_equal(t0[sure], t1[sure])


def test_the_cap_keeps_the_last_trial():
    L = np.log(W8)
    a1, _, t1 = oracle.rejection(L, 1, 3, 2, 5)
    assert np.array_equal(a1, np.arange(8))      # one trial: the own particle
    assert np.all(t1 == 1)
    # a slot stopped by the cap keeps the proposal of its last trial, which is
    # the proposal a longer run tested at that trial
    full, _, tf = oracle.rejection(L, 4096, 3, 2, 5)
    a2, _, t2 = oracle.rejection(L, 2, 3, 2, 5)
    done = tf <= 2
    assert np.array_equal(a2[done], full[done])
    assert np.all(t2 <= 2)
