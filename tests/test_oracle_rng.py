"""Pins of the oracle's random streams (Philox4x32-10 + Box-Muller).

The generator is pinned to things outside the oracle:
  * numpy.random.Philox is Philox4x64-10; the oracle's 64-bit-word Philox is the
    same round/key-schedule code with 64-bit constants and must reproduce it;
  * the published known-answer values of Philox4x32-10 (tests/golden);
  * statistics: uniformity (chi-square) and normality (Kolmogorov-Smirnov,
    moments) of the Box-Muller draws against scipy.
"""
import os

import numpy as np
import pytest
import scipy.stats as st

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(s, 16) for s in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox4x32_known_answers(ctr, key, want):
    got = oracle.philox4x32_10(ctr, key)
    assert [int(g) for g in got] == want


@pytest.mark.parametrize("key", [(0, 0), (12345, 0xDEADBEEF), (2**64 - 1, 7)])
def test_philox4x64_matches_numpy(key):
    # numpy's Philox increments the 256-bit counter before each block, so the
    # i-th block of random_raw comes from counter value start + i + 1.
    start = [3, 0, 0, 0]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(start, dtype=np.uint64))
    raw = bg.random_raw(4 * 6).reshape(6, 4)
    for i in range(6):
        ctr = [start[0] + i + 1, 0, 0, 0]
        got = oracle.philox4x64_10(ctr, key)
        assert [int(v) for v in got] == [int(v) for v in raw[i]]


def test_philox4x64_counter_carry_matches_numpy():
    # Counter words other than the first also enter the rounds: exercise a carry.
    start = [2**64 - 2, 5, 0, 0]
    bg = np.random.Philox(key=np.array([9, 9], dtype=np.uint64),
                          counter=np.array(start, dtype=np.uint64))
    raw = bg.random_raw(8).reshape(2, 4)
    got0 = oracle.philox4x64_10([2**64 - 1, 5, 0, 0], [9, 9])
    got1 = oracle.philox4x64_10([0, 6, 0, 0], [9, 9])
    assert [int(v) for v in got0] == [int(v) for v in raw[0]]
    assert [int(v) for v in got1] == [int(v) for v in raw[1]]


def test_philox_words_key_and_counter_layout():
    seed = 0x0123456789ABCDEF
    got = oracle.philox_words(seed, 7, 3, 11, 1)
    want = oracle.philox4x32_10([7, 3, 11, 1], [seed & 0xFFFFFFFF, seed >> 32])
    assert list(got) == list(want)


def test_uniform53_bits():
    assert oracle.uniform53(0, 0) == 0.0
    assert oracle.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle.uniform53(0x80000000, 0) == 0.5
    # low 11 bits of the second word are discarded
    assert oracle.uniform53(1, 0x7FF) == oracle.uniform53(1, 0)
    assert oracle.uniform53(0, 0x800) == 2.0 ** -53


def _normals(n, seed=0, t=1, stream=0):
    # propagate with drift 0 and sigma 1 from the origin returns the draws
    p = oracle.make_params(n, 64, 64, drift=(0.0, 0.0), sigma=(1.0, 1.0), seed=seed,
                           stream_id=stream)
    return oracle.propagate(p, t, np.zeros(n), np.zeros(n))


def test_normal_pair_is_box_muller_of_the_stream():
    seed, k, t, s = 42, 17, 5, 3
    w = oracle.philox_words(seed, k, t, s, 0)
    ua = oracle.uniform53(int(w[0]), int(w[1]))
    ub = oracle.uniform53(int(w[2]), int(w[3]))
    zx, zy = oracle.normal_pair(seed, k, t, s)
    rho = np.sqrt(-2.0 * np.log1p(-ua))
    assert zx == pytest.approx(rho * np.cos(2 * np.pi * ub), rel=1e-12, abs=1e-12)
    assert zy == pytest.approx(rho * np.sin(2 * np.pi * ub), rel=1e-12, abs=1e-12)


def test_uniform_chi_square():
    n = 200_000
    u = np.array([oracle.u0(1, 0, t) for t in range(n // 100)])  # resampling offsets
    # the particle stream: first word of each block
    zx, zy = _normals(n, seed=7)
    # map normals back to uniforms through the normal CDF; must be U(0,1)
    for v in (zx, zy):
        uu = st.norm.cdf(v)
        hist, _ = np.histogram(uu, bins=50, range=(0, 1))
        chi2 = ((hist - n / 50) ** 2 / (n / 50)).sum()
        assert chi2 < st.chi2.ppf(0.999, 49)
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = ((hist - u.size / 20) ** 2 / (u.size / 20)).sum()
    assert chi2 < st.chi2.ppf(0.999, 19)


def test_box_muller_normality():
    zx, zy = _normals(1_000_000, seed=3, t=2, stream=1)
    for z in (zx, zy):
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
        assert abs(st.kurtosis(z, fisher=False) - 3.0) < 0.03
        assert st.kstest(z, "norm").pvalue > 1e-4
    # the two draws of a pair are uncorrelated
    assert abs(np.corrcoef(zx, zy)[0, 1]) < 5 / np.sqrt(zx.size)


def test_streams_differ_by_particle_step_and_stream():
    a = _normals(1000, seed=0, t=1, stream=0)[0]
    b = _normals(1000, seed=0, t=2, stream=0)[0]
    c = _normals(1000, seed=0, t=1, stream=1)[0]
    d = _normals(1000, seed=1, t=1, stream=0)[0]
    for other in (b, c, d):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.15
    assert len(np.unique(a)) == a.size
