"""Pins of the oracle's Metropolis resampler (Murray, Lee & Jacob 2016) by
properties of the Metropolis chain, not by its formula: zero steps keep every
slot on itself, uniform weights give uniform ancestors, the slots' ancestors
follow the normalised weights once the chains have mixed, a particle that
dominates absorbs a chain at the first proposal of it, and a common shift of
the log-likelihoods changes no decision."""
import numpy as np
import pytest
from scipy import stats

import oracle


def test_zero_steps_keep_every_slot():
    L = np.random.default_rng(0).normal(size=777)
    anc, margin = oracle.metropolis(L, 0, 5, 1, 3)
    assert np.array_equal(anc, np.arange(777))
    assert np.all(margin == 1.0)


def test_uniform_weights_give_uniform_ancestors():
    n = 200_000
    anc, _ = oracle.metropolis(np.zeros(n), 7, 11, 0, 1)
    counts = np.bincount(anc // (n // 50), minlength=50)
    assert stats.chisquare(counts).pvalue > 1e-4
    # every proposal is accepted: no slot stays on itself except by chance
    assert np.mean(anc == np.arange(n)) < 1e-3


def test_mixed_chains_follow_the_normalised_weights():
    # 8 particles with weights 1..8 (normalised), many independent steps t:
    # each slot's ancestor is one draw from the chain after B = 40 steps,
    # whose distance to the weights is below (1 - min_ratio)^B ~ 1e-6 here
    w = np.arange(1, 9, dtype=float)
    L = np.log(w)
    draws = np.concatenate([oracle.metropolis(L, 40, 3, 2, t)[0] for t in range(1, 6001)])
    counts = np.bincount(draws, minlength=8)
    expected = draws.size * w / w.sum()
    assert stats.chisquare(counts, expected).pvalue > 1e-4


def test_a_dominant_particle_absorbs_the_chain():
    # L = -1000 everywhere but particle h: a chain moves to h at its first
    # proposal of h and never leaves; among light particles it moves freely.
    n, B, h = 4096, 16, 1234
    L = np.full(n, -1000.0)
    L[h] = 0.0
    ends = []
    for t in range(1, 41):
        anc, _ = oracle.metropolis(L, B, 9, 4, t)
        ends.append(anc)
    ends = np.concatenate(ends)
    p = 1.0 - (1.0 - 1.0 / n) ** B          # P(h proposed at least once)
    hits = np.sum(ends == h)
    sd = np.sqrt(ends.size * p * (1 - p))
    assert abs(hits - ends.size * p) < 5 * sd


def test_a_common_shift_changes_no_decision():
    rng = np.random.default_rng(2)
    L = rng.normal(scale=3.0, size=5000)
    a0, m0 = oracle.metropolis(L, 24, 1, 7, 2)
    a1, m1 = oracle.metropolis(L + 17.25, 24, 1, 7, 2)
    sure = (m0 > 1e-9) & (m1 > 1e-9)
    assert sure.mean() > 0.99
    assert np.array_equal(a0[sure], a1[sure])
