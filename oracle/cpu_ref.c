/*
 * Plain C, FP64 statement of InfraredGP's feed-forward propagation.
 * TEST INFRASTRUCTURE ONLY: called by the test suite and the benchmark's
 * CPU-baseline leg through oracle/cref.py; never linked into the product.
 *
 * Same mathematics as oracle/ffp.py, for graphs too large for the NumPy
 * version to finish in seconds.  Rows are split over OpenMP threads; nothing
 * else is blocked, fused or reordered.
 *
 *   D_tau     Eq. (1) for tau <= 0 (literal form), D + tau I for tau > 0
 *   s_i       (D_tau)_ii^{-1/2}
 *   Z^(0)     N(0, 1/d): Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 *             counter (i+1, c/4, 0, 0); Box-Muller on words (0, 1) gives
 *             columns 4q, 4q+1 (cos, sin), on words (2, 3) columns 4q+2, 4q+3
 *   hop       Y = theta Z + alpha S A S Z        (Eq. (3))
 *   layer     Z = ZNorm(tanh(Y)), column z-score with divisor N - ddof (Eq. (4))
 *   output    sigma(Z^(K))                       (Eq. (4))
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t mulhilo64(uint64_t a, uint64_t b, uint64_t *hi)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    return (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], uint64_t k0, uint64_t k1, uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t hi0, hi1;
        uint64_t lo0 = mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0);
        uint64_t lo1 = mulhilo64(0xCA5A826395121157ULL, c2, &hi1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u53(uint64_t o) { return ((double)(o >> 11) + 0.5) * 0x1p-53; }

void oracle_gaussian_input(int64_t N, int32_t d, uint64_t seed, double *X)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int32_t c = 0; c < d; ++c) {
            uint64_t ctr[4] = {(uint64_t)i + 1, (uint64_t)(c / 4), 0, 0}, o[4];
            oracle_philox4x64_10(ctr, seed, 0, o);
            const int j = c % 4;
            const double ua = u53(j < 2 ? o[0] : o[2]);
            const double ub = u53(j < 2 ? o[1] : o[3]);
            const double r = sqrt(-2.0 * log(ua)), phi = 2.0 * M_PI * ub;
            const double z = (j % 2 == 0) ? r * cos(phi) : r * sin(phi);
            X[i * d + c] = z / sqrt((double)d);
        }
    }
}

void oracle_scales(int64_t N, const int64_t *rowptr, double tau, double eps, double *s)
{
    for (int64_t i = 0; i < N; ++i) {
        double deg = (double)(rowptr[i + 1] - rowptr[i]);
        double dt;
        if (tau > 0) dt = deg + tau;
        else {
            double m = fabs(tau) < deg - eps ? fabs(tau) : deg - eps;
            dt = deg - m;
        }
        s[i] = 1.0 / sqrt(dt);
    }
}

/* out = sigma(Z^(K)) with Z^(0) = X; out may alias nothing. */
int oracle_ffp(int64_t N, const int64_t *rowptr, const int64_t *colidx, double tau, int32_t K,
               int32_t d, const double *X, double alpha, double theta, double eps, int32_t ddof,
               double *out)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *Z = (double *)malloc(sizeof(double) * (size_t)(N * d > 0 ? N * d : 1));
    double *Y = (double *)malloc(sizeof(double) * (size_t)(N * d > 0 ? N * d : 1));
    double *mu = (double *)calloc((size_t)d, sizeof(double));
    double *sd = (double *)calloc((size_t)d, sizeof(double));
    if (!s || !Z || !Y || !mu || !sd) {
        free(s); free(Z); free(Y); free(mu); free(sd);
        return -1;
    }
    oracle_scales(N, rowptr, tau, eps, s);
    memcpy(Z, X, sizeof(double) * (size_t)(N * d));

    for (int32_t l = 0; l < K; ++l) {
        /* Y = tanh(theta Z + alpha S A S Z) */
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i) {
            double *y = Y + i * d;
            for (int32_t c = 0; c < d; ++c) y[c] = 0.0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                int64_t j = colidx[e];
                for (int32_t c = 0; c < d; ++c) y[c] += s[j] * Z[j * d + c];
            }
            for (int32_t c = 0; c < d; ++c)
                y[c] = tanh(theta * Z[i * d + c] + alpha * s[i] * y[c]);
        }
        /* column mean and standard deviation */
        for (int32_t c = 0; c < d; ++c) { mu[c] = 0.0; sd[c] = 0.0; }
        for (int64_t i = 0; i < N; ++i)
            for (int32_t c = 0; c < d; ++c) mu[c] += Y[i * d + c];
        for (int32_t c = 0; c < d; ++c) mu[c] /= (double)N;
        for (int64_t i = 0; i < N; ++i)
            for (int32_t c = 0; c < d; ++c) {
                double t = Y[i * d + c] - mu[c];
                sd[c] += t * t;
            }
        for (int32_t c = 0; c < d; ++c)
            sd[c] = (N - ddof > 0) ? sqrt(sd[c] / (double)(N - ddof)) : 0.0;
        /* Z = ZNorm(Y); a column with zero spread becomes zero */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            for (int32_t c = 0; c < d; ++c)
                Z[i * d + c] = sd[c] > 0.0 ? (Y[i * d + c] - mu[c]) / sd[c] : 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N * d; ++i) out[i] = 1.0 / (1.0 + exp(-Z[i]));

    free(s); free(Z); free(Y); free(mu); free(sd);
    return 0;
}
