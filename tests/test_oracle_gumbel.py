"""Pins of the oracle's Gumbel-max multinomial resampler by properties of the
scheme, not by its formula: each slot's ancestor is a draw from the
normalised weights (so uniform log weights give uniform ancestors and a
weight vector is reproduced in distribution), slots draw independently, a
common shift of the log weights changes no choice, and a particle that
outweighs the rest by far more than the Gumbel noise can span takes every
slot."""
import numpy as np
from scipy import stats

import oracle


def test_ancestors_follow_the_normalised_weights():
    w = np.array([1, 2, 3, 4, 5, 6, 7, 8], dtype=float)
    L = np.log(w) + 3.0
    draws = np.concatenate([oracle.gumbel_max(L, 5, 1, t)[0] for t in range(1, 4001)])
    expected = draws.size * w / w.sum()
    assert stats.chisquare(np.bincount(draws, minlength=8), expected).pvalue > 1e-4


def test_uniform_weights_give_uniform_independent_ancestors():
    n = 3000
    anc, _ = oracle.gumbel_max(np.zeros(n), 2, 3, 1)
    counts = np.bincount(anc, minlength=n)
    # multinomial(n, 1/n): the number of particles with c offspring is about
    # n * Poisson(1) pmf(c)
    occ = np.bincount(counts, minlength=6)[:6]
    expected = n * stats.poisson.pmf(np.arange(6), 1.0)
    assert stats.chisquare(occ[:5], expected[:5] * occ[:5].sum() / expected[:5].sum()).pvalue > 1e-4


def test_a_common_shift_changes_no_choice():
    rng = np.random.default_rng(4)
    L = rng.normal(scale=2.0, size=1500)
    a0, m0 = oracle.gumbel_max(L, 8, 2, 5)
    a1, m1 = oracle.gumbel_max(L - 123.5, 8, 2, 5)
    sure = (m0 > 1e-9) & (m1 > 1e-9)
    assert sure.mean() > 0.999
    assert np.array_equal(a0[sure], a1[sure])


def test_a_dominant_particle_takes_every_slot():
    n, h = 2000, 777
    L = np.full(n, -500.0)
    L[h] = 0.0
    anc, margin = oracle.gumbel_max(L, 1, 0, 3)
    assert np.all(anc == h) and np.all(margin > 400.0)
