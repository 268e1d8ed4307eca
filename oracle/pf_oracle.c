/*
 * pf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, double-precision CPU reference of the per-frame
 * sampling-importance-resampling (SIR) step of the half-precision particle
 * filter paper (Schieffer et al., "Boosting the Performance of Object Tracking
 * with a Half-Precision Particle Filter on GPU", arXiv:2308.00763).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this code.  The product (the HIP library) shares nothing with it: no
 * header, no helper, no table.  Every function here is written to be checked
 * by eye against the paper; there is no blocking, fusion or reordering beyond
 * what the paper's definitions state.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared pf_oracle.c -lm
 * (-ffp-contract=off keeps every a*b+c as two roundings, as written.)
 *
 * Readings of the paper taken here (each is justified where it is used):
 *   - Eq. (2) prints the mean as "2.0 + y"; the tracked object moves toward
 *     y = 0 (Sec. 5, verification paragraph), so the drift is a parameter and
 *     the workloads use d_y = -2.
 *   - Eq. (3) prints no sum; the likelihood sums the per-pixel term over the
 *     pixel set around the particle and divides by 50 * N_d (MEAN) -- or by 50
 *     only (SUM, a flag).
 *   - The pixel set is the strict disk dx^2 + dy^2 < r^2.
 *   - Pixel rounding is half-up: cell = floor(v + 1/2); pixels outside the
 *     frame are clamped to the nearest edge.
 *   - Random numbers come from the counter-based Philox4x32-10 generator
 *     (Salmon et al., SC'11) and Box-Muller; the paper draws in double and
 *     converts (Sec. 4, after Eq. (2)); the counter layout is this implementation's.
 *
 * parity pinned: Philox against numpy's Philox4x64-10 (same code, 64-bit
 * words) and known-answer values; every other function by closed forms,
 * invariants, brute force and a Kalman filter (see tests/).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox-4xW-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11, Sec. 3).  One round maps the counter words
 * (X0, X1, X2, X3) with key (K0, K1) to
 *     (hi(M1*X2) ^ X1 ^ K0,  lo(M1*X2),  hi(M0*X0) ^ X3 ^ K1,  lo(M0*X0))
 * and the key is bumped by the Weyl constants between rounds.  The 32- and
 * 64-bit word versions are the same function with different constants; the
 * 64-bit one is exposed so a test can compare it with numpy.random.Philox. */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        if (round > 0) { k0 += W0; k1 += W1; }
        mulhilo32(M0, x0, &hi0, &lo0);
        mulhilo32(M1, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        if (round > 0) { k0 += W0; k1 += W1; }
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout of the random streams (this implementation's choice; the paper only
 * says one seed is shared across precisions, Sec. 5):
 *   particle draw of particle k at step t: ctr = (k, t, stream_id, 0)
 *   resampling offset of step t:           ctr = (0, t, stream_id, 1)
 * key = (low 32 bits of seed, high 32 bits of seed). */
void or_philox_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* A uniform double in [0, 1) made of 53 random bits: the 32 bits of `hi`
 * followed by the top 21 bits of `lo`, scaled by 2^-53. */
double or_uniform53(uint32_t hi, uint32_t lo)
{
    uint64_t bits = ((uint64_t)hi << 21) | ((uint64_t)lo >> 11);
    return (double)bits * 0x1.0p-53;
}

/* Two independent standard normals by the Box-Muller transform (Box & Muller,
 * 1958): rho = sqrt(-2 ln(1 - u_a)), z_x = rho cos(2 pi u_b), z_y = rho
 * sin(2 pi u_b).  1 - u_a lies in (0, 1], so the logarithm is finite. */
void or_normal_pair(uint64_t seed, uint32_t k, uint32_t t, uint32_t stream_id,
                    double *zx, double *zy)
{
    uint32_t w[4];
    or_philox_words(seed, k, t, stream_id, 0u, w);
    double ua = or_uniform53(w[0], w[1]);
    double ub = or_uniform53(w[2], w[3]);
    double rho = sqrt(-2.0 * log(1.0 - ua));
    double ang = 6.283185307179586 * ub; /* 2*pi rounded to double */
    *zx = rho * cos(ang);
    *zy = rho * sin(ang);
}

/* The resampling offset u0 in [0, 1) of step t. */
double or_u0(uint64_t seed, uint32_t stream_id, uint32_t t)
{
    uint32_t w[4];
    or_philox_words(seed, 0u, t, stream_id, 1u, w);
    return or_uniform53(w[0], w[1]);
}

/* ------------------------------------------------------------------ */
/* The pixel set around a particle: all integer offsets (dx, dy) with
 * dx^2 + dy^2 < r^2, listed row by row (dy ascending, then dx ascending).
 * Returns the count N_d; writes at most `cap` offsets. */
int or_disk(int r, int *dx, int *dy, int cap)
{
    int n = 0;
    for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i)
            if (i * i + j * j < r * r) {
                if (n < cap) { dx[n] = i; dy[n] = j; }
                ++n;
            }
    return n;
}

typedef struct {
    int64_t n;          /* particles */
    int32_t width;      /* frame columns (x) */
    int32_t height;     /* frame rows (y) */
    int32_t radius;     /* disk radius r */
    int32_t fg, bg;     /* foreground / background intensity (228, 100) */
    int32_t lik_norm;   /* 0: divide by kappa * N_d (MEAN); 1: by kappa (SUM) */
    double kappa;       /* 50 */
    double drift_x, drift_y;  /* mean displacement per frame */
    double sigma_x, sigma_y;  /* transition standard deviations */
    uint64_t seed;
    uint32_t stream_id;
} or_params;

/* Propagation (Sec. 4, Eq. (1)-(2)): every particle moves by
 * x <- x + (d_x + sigma_x z_x), y <- y + (d_y + sigma_y z_y), with the
 * normals of its own counter (k, t, stream_id, 0).  In place. */
void or_propagate(const or_params *p, uint32_t t, double *x, double *y)
{
    for (int64_t k = 0; k < p->n; ++k) {
        double zx, zy;
        or_normal_pair(p->seed, (uint32_t)k, t, p->stream_id, &zx, &zy);
        x[k] = x[k] + (p->drift_x + p->sigma_x * zx);
        y[k] = y[k] + (p->drift_y + p->sigma_y * zy);
    }
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Log-likelihood of one particle (Sec. 4, Eq. (3), with the sum over the
 * disk written out): the particle's pixel is c = (floor(x + 1/2),
 * floor(y + 1/2)); over every disk offset the integer term
 * (I - bg)^2 - (I - fg)^2 is summed exactly, then divided once by
 * kappa * N_d (MEAN) or kappa (SUM).  Eq. (4) is the same quantity with the
 * divisor moved inside the squares, so it is not computed separately. */
double or_likelihood_one(const or_params *p, const uint8_t *frame, int64_t pitch,
                         double x, double y)
{
    int r = p->radius;
    int64_t cx = (int64_t)floor(x + 0.5);
    int64_t cy = (int64_t)floor(y + 0.5);
    int64_t s = 0;
    int nd = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            if (dx * dx + dy * dy >= r * r) continue;
            int64_t row = clampi(cy + dy, 0, p->height - 1);
            int64_t col = clampi(cx + dx, 0, p->width - 1);
            int64_t I = frame[row * pitch + col];
            s += (I - p->bg) * (I - p->bg) - (I - p->fg) * (I - p->fg);
            ++nd;
        }
    double denom = p->lik_norm == 0 ? p->kappa * (double)nd : p->kappa;
    return (double)s / denom;
}

void or_likelihood(const or_params *p, const uint8_t *frame, int64_t pitch,
                   const double *x, const double *y, double *L)
{
    for (int64_t k = 0; k < p->n; ++k)
        L[k] = or_likelihood_one(p, frame, pitch, x[k], y[k]);
}

/* Weighting, normalising, estimate and systematic resampling (Sec. 4,
 * Eq. (5) and the normalizing/resampling paragraphs), given the
 * log-likelihoods L of the propagated particles (x, y):
 *   M      = max_k L_k
 *   wh_k   = w_prev_k * exp(L_k - M)                    (Eq. (5))
 *   P_k    = wh_0 + ... + wh_k  (summed left to right),  Z = P_{n-1}
 *   w_k    = wh_k / Z,   C_k = P_k / Z   (so C_{n-1} = 1)
 *   est    = (sum_k w_k x_k, sum_k w_k y_k)  (before resampling)
 *   u_j    = (j + u0) / n  -- one point in each of the n strata of [0, 1)
 *   a_j    = the first i with C_i >= u_j (n - 1 if none)
 *   out_j  = (x_{a_j}, y_{a_j})
 * Outputs that are NULL are not written (cdf, anc, w_norm may be NULL). */
void or_reweight_resample(int64_t n, const double *L, const double *w_prev,
                          const double *x, const double *y, double u0,
                          double *w_norm, double *cdf, int32_t *anc,
                          double *x_out, double *y_out, double est[2])
{
    double M = L[0];
    for (int64_t k = 1; k < n; ++k)
        if (L[k] > M) M = L[k];

    double *wh = (double *)malloc((size_t)n * sizeof(double));
    double *P = (double *)malloc((size_t)n * sizeof(double));
    double run = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        wh[k] = w_prev[k] * exp(L[k] - M);
        run = run + wh[k];
        P[k] = run;
    }
    double Z = P[n - 1];

    double ex = 0.0, ey = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double w = wh[k] / Z;
        if (w_norm) w_norm[k] = w;
        if (cdf) cdf[k] = P[k] / Z;
        ex = ex + w * x[k];
        ey = ey + w * y[k];
    }
    est[0] = ex;
    est[1] = ey;

    /* a_j is non-decreasing in j because u_j increases, so the search for
     * a_j may start at a_{j-1}. */
    int64_t i = 0;
    for (int64_t j = 0; j < n; ++j) {
        double uj = ((double)j + u0) / (double)n;
        while (i < n - 1 && P[i] / Z < uj) ++i;
        if (anc) anc[j] = (int32_t)i;
        if (x_out) x_out[j] = x[i];
        if (y_out) y_out[j] = y[i];
    }
    free(wh);
    free(P);
}

/* ------------------------------------------------------------------ */
/* Metropolis resampling (Murray, Lee & Jacob, "Parallel resampling in the
 * particle filter", J. Comput. Graph. Stat. 2016), the scan-free resampler
 * among the related work the paper cites (Sec. 3): slot j runs its own
 * Metropolis chain of B steps over the particle indices, whose stationary
 * distribution is the normalised weights.  The chain starts at k = j; each
 * step proposes a particle i uniformly and moves there with probability
 * min(1, w_i / w_k) = min(1, exp(L_i - L_k)).  Only ratios of weights enter:
 * no maximum, sum or cumulative distribution.
 * Random numbers of slot j at step t (this implementation's layout): steps b = 2m and
 * 2m + 1 share ctr = (j, t, stream_id, 2 + m); step 2m uses words 0 and 1,
 * step 2m + 1 words 2 and 3; the first picks i = floor(word * n / 2^32), the
 * second gives u = (word + 1/2) 2^-32 in (0, 1), and the move is taken when
 * L_i >= L_k or u <= exp(L_i - L_k).
 * margin (optional, length n): for slot j the smallest |u - exp(L_i - L_k)|
 * over its chain's comparisons with L_i < L_k (1 if none), so a comparison
 * with another implementation can tell the decisions rounding could flip. */
void or_metropolis(int64_t n, const double *L, int32_t B, uint64_t seed, uint32_t stream_id,
                   uint32_t t, int32_t *anc, double *margin)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t k = j;
        double mg = 1.0;
        uint32_t w[4] = {0, 0, 0, 0};
        for (int32_t b = 0; b < B; ++b) {
            if (b % 2 == 0) or_philox_words(seed, (uint32_t)j, t, stream_id, 2u + (uint32_t)(b / 2), w);
            uint32_t wi = (b % 2 == 0) ? w[0] : w[2];
            uint32_t wu = (b % 2 == 0) ? w[1] : w[3];
            int64_t i = (int64_t)(((uint64_t)wi * (uint64_t)n) >> 32);
            if (L[i] >= L[k]) {
                k = i;
                continue;
            }
            double ratio = exp(L[i] - L[k]);
            double u = ((double)wu + 0.5) * 0x1.0p-32;
            double d = fabs(u - ratio);
            if (d < mg) mg = d;
            if (u <= ratio) k = i;
        }
        anc[j] = (int32_t)k;
        if (margin) margin[j] = mg;
    }
}

/* ------------------------------------------------------------------ */
/* Rejection resampling (Murray, Lee & Jacob 2016, the other scan-free
 * resampler of the related work the paper cites, Sec. 3): slot j first
 * proposes its own particle c = j; a proposal c is accepted with probability
 * w_c / w_max = exp(L_c - M), M = max_k L_k; after a rejection the next
 * proposal is a particle drawn uniformly.  It needs the maximum but no sum or
 * cumulative distribution.  Each particle's expected offspring count is
 * exactly N w_i / sum(w): P(a_j = i) = [i = j] r_j + (1 - r_j) w_i / sum(w)
 * with r_j = w_j / w_max, and summing over j gives N w_i / sum(w).  The
 * expected number of trials of slot j is 1 + (1 - r_j) N w_max / sum(w).
 * At most `cap` trials: a slot that rejects all of them keeps the particle
 * of its last trial (a bias the cap bounds).
 * Random numbers of slot j at step t (this implementation's layout): trials m = 2q
 * and 2q + 1 share ctr = (j, t, stream_id, 2 + q); trial 2q uses words 0
 * and 1, trial 2q + 1 words 2 and 3; the first word gives u = (word + 1/2)
 * 2^-32, the test u <= exp(L_c - M), and the second the next proposal
 * floor(word * n / 2^32).
 * margin (optional): for slot j the smallest |u - exp(L_c - M)| over its
 * trials; trials (optional): the number of trials slot j took. */
void or_rejection(int64_t n, const double *L, int32_t cap, uint64_t seed, uint32_t stream_id,
                  uint32_t t, int32_t *anc, double *margin, int32_t *trials)
{
    double M = -INFINITY;
    for (int64_t k = 0; k < n; ++k)
        if (L[k] > M) M = L[k];
    for (int64_t j = 0; j < n; ++j) {
        int64_t c = j;
        double mg = 1.0;
        uint32_t w[4] = {0, 0, 0, 0};
        int32_t m = 0;
        for (; m < cap; ++m) {
            if (m % 2 == 0) or_philox_words(seed, (uint32_t)j, t, stream_id, 2u + (uint32_t)(m / 2), w);
            uint32_t wu = (m % 2 == 0) ? w[0] : w[2];
            uint32_t wi = (m % 2 == 0) ? w[1] : w[3];
            double u = ((double)wu + 0.5) * 0x1.0p-32;
            double r = exp(L[c] - M);
            double d = fabs(u - r);
            if (d < mg) mg = d;
            if (u <= r) break;
            if (m + 1 < cap) c = (int64_t)(((uint64_t)wi * (uint64_t)n) >> 32);
        }
        anc[j] = (int32_t)c;
        if (margin) margin[j] = mg;
        if (trials) trials[j] = m < cap ? m + 1 : cap;
    }
}

/* ------------------------------------------------------------------ */
/* Multinomial resampling by the Gumbel-max scheme (the alternative the
 * paper weighs in Sec. 4, numerical-stability paragraph): slot i takes
 * a_i = argmax_j (L_j + G_ij) with G_ij independent standard Gumbel
 * variables, so P(a_i = j) is the normalised weight of j; it works on the
 * unnormalised log weights (no maximum, normaliser or cumulative
 * distribution) and costs n^2 noise draws.
 * G_ij = -ln(-ln u), u = (word + 1/2) 2^-32, word j mod 4 of Philox at
 * counter (floor(j / 4), i, t, stream_id) with key (low 32 bits of seed,
 * high 32 bits of seed xor 0x47756D62) -- a key of its own, so these words
 * never coincide with the other streams of the filter.  Ties go to the lower
 * index.  margin (optional): for slot i the gap between the best and the
 * second-best score. */
void or_gumbel_max(int64_t n, const double *L, uint64_t seed, uint32_t stream_id, uint32_t t,
                   int32_t *anc, double *margin)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x47756D62u};
    for (int64_t i = 0; i < n; ++i) {
        double best = -INFINITY, second = -INFINITY;
        int64_t arg = 0;
        uint32_t w[4] = {0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j % 4 == 0) {
                uint32_t ctr[4] = {(uint32_t)(j / 4), (uint32_t)i, t, stream_id};
                or_philox4x32_10(ctr, key, w);
            }
            double u = ((double)w[j % 4] + 0.5) * 0x1.0p-32;
            double g = -log(-log(u));
            double v = L[j] + g;
            if (v > best) {
                second = best;
                best = v;
                arg = j;
            } else if (v > second) {
                second = v;
            }
        }
        anc[i] = (int32_t)arg;
        if (margin) margin[i] = best - second;
    }
}

/* One whole SIR step t (t = 1, 2, ...) on frame `frame`.
 * In:  x, y -- the particles after the previous resampling (all weights 1/n).
 * Out: x, y -- the particles after this step's resampling;
 *      optional per-particle diagnostics of this step (NULL to skip):
 *      x_prop, y_prop (propagated), L, w_norm (before resampling), anc;
 *      est -- the weighted position estimate before resampling. */
void or_step(const or_params *p, uint32_t t, const uint8_t *frame, int64_t pitch,
             double *x, double *y, double *x_prop, double *y_prop, double *L,
             double *w_norm, int32_t *anc, double est[2])
{
    int64_t n = p->n;
    double *xp = (double *)malloc((size_t)n * sizeof(double));
    double *yp = (double *)malloc((size_t)n * sizeof(double));
    double *LL = (double *)malloc((size_t)n * sizeof(double));
    double *wp = (double *)malloc((size_t)n * sizeof(double));
    memcpy(xp, x, (size_t)n * sizeof(double));
    memcpy(yp, y, (size_t)n * sizeof(double));
    or_propagate(p, t, xp, yp);
    or_likelihood(p, frame, pitch, xp, yp, LL);
    /* Resampling happens every frame, so every previous weight is 1/n. */
    for (int64_t k = 0; k < n; ++k) wp[k] = 1.0 / (double)n;
    double u0 = or_u0(p->seed, p->stream_id, t);
    or_reweight_resample(n, LL, wp, xp, yp, u0, w_norm, NULL, anc, x, y, est);
    if (x_prop) memcpy(x_prop, xp, (size_t)n * sizeof(double));
    if (y_prop) memcpy(y_prop, yp, (size_t)n * sizeof(double));
    if (L) memcpy(L, LL, (size_t)n * sizeof(double));
    free(xp); free(yp); free(LL); free(wp);
}

/* Initialisation and a run over frames 1..T-1 of a video (frames of
 * height*pitch bytes each, back to back): all particles start at (x0, y0)
 * with weight 1/n; step t uses frame t.  est_out holds 2*T doubles: the
 * estimate of frame 0 is (x0, y0), then one estimate per step.
 * x, y (length n) receive the final particles. */
void or_run(const or_params *p, const uint8_t *video, int64_t pitch, int32_t T,
            double x0, double y0, double *x, double *y, double *est_out)
{
    for (int64_t k = 0; k < p->n; ++k) { x[k] = x0; y[k] = y0; }
    est_out[0] = x0;
    est_out[1] = y0;
    for (int32_t t = 1; t < T; ++t) {
        const uint8_t *frame = video + (int64_t)t * (int64_t)p->height * pitch;
        or_step(p, (uint32_t)t, frame, pitch, x, y, NULL, NULL, NULL, NULL, NULL,
                &est_out[2 * t]);
    }
}
