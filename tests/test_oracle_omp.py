"""The OpenMP timing build of the oracle (pf_oracle_omp.c) against the
sequential oracle it parallelises: the same propagated particles and
likelihoods, weights and estimate equal up to the rounding of a different
summation order, and the same ancestors except where a stratum point lies
within that rounding of a cumulative weight.  It only times the oracle on
many cores; this test makes sure what it times is the same step."""
import numpy as np
import pytest

import oracle
import pfsynth


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_omp_step_equals_sequential_step(threads):
    w = pfsynth.WORKLOADS["disk128_n1000"]
    n = 4099  # not a multiple of the thread count
    vid = pfsynth.workload_video(w, frames=4)
    p = oracle.make_params(n, w.width, w.height, radius=w.radius, drift=w.drift, sigma=w.sigma,
                           seed=w.filter_seed)
    x0, y0 = vid.centres[0]
    x = np.full(n, x0)
    y = np.full(n, y0)
    st = oracle.OmpStepper(p, x, y, threads=threads)
    for t in (1, 2, 3):
        ref = oracle.step(p, t, vid.frames[t], x, y)
        est = st.step(t, vid.frames[t])
        assert st.threads == threads
        assert np.array_equal(st.xp, ref["x_prop"]) and np.array_equal(st.yp, ref["y_prop"])
        Z = st.P[-1]
        np.testing.assert_allclose(st.L / Z, ref["w"], rtol=0, atol=1e-13)
        np.testing.assert_allclose(est, ref["est"], rtol=0, atol=1e-9)
        # ancestors: the state after resampling is the ancestors' positions;
        # a slot may differ only where its stratum point is within 1e-12 of
        # the cumulative weight at the boundary
        cdf = np.cumsum(ref["w"])
        u0 = oracle.u0(w.filter_seed, 0, t)
        u = (np.arange(n) + u0) / n
        same = (st.x == ref["x"]) & (st.y == ref["y"])
        for j in np.flatnonzero(~same):
            assert np.min(np.abs(cdf - u[j])) <= 1e-12, (t, j)
        x, y = ref["x"], ref["y"]
        st.x[:] = x
        st.y[:] = y
