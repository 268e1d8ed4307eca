/*
 * pf_oracle_omp.c -- TEST INFRASTRUCTURE ONLY (timing build).
 *
 * The FP64 oracle step of pf_oracle.c spread over the host's cores with
 * OpenMP, used only to time the oracle on every core the host gives it (the
 * CPU baseline of the benchmark).  Parity tests use the sequential build.
 *
 * It runs the same per-particle functions as the sequential oracle (this
 * file includes pf_oracle.c): the draws, the propagation (Sec. 4,
 * Eq. (1)-(2)) and the disk likelihood (Eq. (3)) are identical particle by
 * particle.  Only the sums change order: the maximum, the normaliser and the
 * estimate are formed as per-thread partial results over contiguous particle
 * ranges, combined in thread order, and the cumulative weights are a
 * two-pass parallel scan (each thread's local prefix sums, then the carried
 * totals of the threads before it).  So its weights, estimate and ancestors
 * agree with the sequential oracle up to rounding (an ancestor can differ
 * only where a stratum point is within rounding of a cumulative weight), not
 * bit for bit; a CPU test checks that agreement.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared pf_oracle_omp.c -lm
 */
#include <omp.h>

#include "pf_oracle.c"

/* One whole SIR step t on `frame` (the sequential or_step's contract):
 * x, y in: the particles after the previous resampling; out: after this
 * step's resampling.  xp, yp, L, P are caller-provided work arrays of n
 * doubles (on return: the propagated positions, the unnormalised weights and
 * the cumulative weights); est receives the estimate before resampling.
 * Returns the number of threads that ran the step. */
int or_step_omp(const or_params *p, uint32_t t, const uint8_t *frame, int64_t pitch,
                double *x, double *y, double *xp, double *yp, double *L, double *P,
                double est[2])
{
    const int64_t n = p->n;
    const double u0 = or_u0(p->seed, p->stream_id, t);
    int nth_used = 1;
    /* per thread: maximum, total weight, carried offset, estimate sums */
    double *part = (double *)calloc((size_t)omp_get_max_threads() * 5, sizeof(double));
    double M = -INFINITY, Z = 0.0;
#pragma omp parallel
    {
        const int nth = omp_get_num_threads(), me = omp_get_thread_num();
        const int64_t lo = n * me / nth, hi = n * (me + 1) / nth;
#pragma omp single
        nth_used = nth;
        /* propagate and score (O3-O5) */
        double m = -INFINITY;
        for (int64_t k = lo; k < hi; ++k) {
            double zx, zy;
            or_normal_pair(p->seed, (uint32_t)k, t, p->stream_id, &zx, &zy);
            xp[k] = x[k] + (p->drift_x + p->sigma_x * zx);
            yp[k] = y[k] + (p->drift_y + p->sigma_y * zy);
            L[k] = or_likelihood_one(p, frame, pitch, xp[k], yp[k]);
            if (L[k] > m) m = L[k];
        }
        part[5 * me] = m;
#pragma omp barrier
#pragma omp single
        {
            for (int i = 0; i < nth; ++i)
                if (part[5 * i] > M) M = part[5 * i];
        }
        /* weights (previous weights 1/n) and the thread's local prefix sums (O6-O8) */
        const double wprev = 1.0 / (double)n;
        double run = 0.0;
        for (int64_t k = lo; k < hi; ++k) {
            L[k] = wprev * exp(L[k] - M);  /* L now holds the weight */
            run = run + L[k];
            P[k] = run;
        }
        part[5 * me + 1] = run;
#pragma omp barrier
#pragma omp single
        {
            double c = 0.0;
            for (int i = 0; i < nth; ++i) {
                part[5 * i + 2] = c;
                c = c + part[5 * i + 1];
            }
            Z = c;
        }
        const double carry = part[5 * me + 2];
        double sx = 0.0, sy = 0.0;
        for (int64_t k = lo; k < hi; ++k) {
            const double w = L[k] / Z;
            P[k] = carry + P[k];
            sx = sx + w * xp[k];
            sy = sy + w * yp[k];
        }
        part[5 * me + 3] = sx;
        part[5 * me + 4] = sy;
#pragma omp barrier
        /* systematic resampling of the thread's slot range (O10-O12): the
         * first ancestor by binary search, then a forward walk */
        if (lo < hi) {
            double u = ((double)lo + u0) / (double)n;
            int64_t a = 0, b = n - 1;
            while (a < b) {
                const int64_t mid = a + (b - a) / 2;
                if (P[mid] / Z < u) a = mid + 1; else b = mid;
            }
            int64_t i = a;
            for (int64_t j = lo; j < hi; ++j) {
                u = ((double)j + u0) / (double)n;
                while (i < n - 1 && P[i] / Z < u) ++i;
                x[j] = xp[i];
                y[j] = yp[i];
            }
        }
    }
    double ex = 0.0, ey = 0.0;
    for (int i = 0; i < nth_used; ++i) {
        ex = ex + part[5 * i + 3];
        ey = ey + part[5 * i + 4];
    }
    est[0] = ex;
    est[1] = ey;
    free(part);
    return nth_used;
}

/* Threads for the following steps (0: leave OpenMP's default). */
void or_omp_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int or_omp_max_threads(void)
{
    return omp_get_max_threads();
}
