/*
 * FP64 CPU oracle for the rejection-ABC hot path of Kulkarni, Krell, Nabarro
 * and Moritz, "Hardware-accelerated Simulation-based Inference of Stochastic
 * Epidemiology Models for COVID-19" (arXiv 2012.14332).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header or constant table with the HIP implementation; the two agree only
 * because both follow the same written definitions.
 *
 * Deliberately plain and slow: one trajectory at a time, every quantity in
 * double precision (counts in int64), the operations in the order the paper
 * states them, no blocking or fusion. OpenMP only splits independent
 * samples across host threads.
 *
 * Definitions followed (paper section / equation):
 *   theta = [alpha0, alpha, n, beta, gamma, delta, eta, kappa]     eq. (1)
 *   prior  U(lo, hi), paper default lo = 0, hi = [1,100,2,1,1,1,1,2] eq. (2)
 *   state  X = [S, I, A, R, D, Ru]                                 eq. (3)
 *   init   Ru = 0, I0 = kappa*A0, S = P - (A0 + R0 + D0 + I0)       Sec. 2.1
 *   g      = alpha0 + alpha / (1 + (A+R+D)^n)                      eq. (4)
 *   h      = (g S I / P, gamma I, beta A, delta A, beta eta I)      eq. (5)
 *   draw   normal with mean h, then floor                          Sec. 2.1
 *   update S->I, I->A, A->R, A->D, I->Ru in the order of h          Sec. 2.1
 *   dist   Euclidean distance over the observed A, R, D series     Sec. 2.2
 *   accept dist <= eps                                             Sec. 2.2, eq. (7)
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes of the repository):
 *   - noise standard deviation sqrt(h) (Poisson-matched variance h); the
 *     literal "variance sqrt(h)" (standard deviation h^(1/4)) is mode 1;
 *   - each draw is clamped to [0, what its source compartment still holds
 *     at the start of the day after earlier outflows in h order];
 *   - I0 = floor(kappa * A0), limited to P - A0 - R0 - D0 so that S >= 0;
 *   - one step per day; the distance covers days 1..T;
 *   - distance on log1p counts (mode 0) or on raw counts (mode 1).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), with
 *   key     = (seed mod 2^32, seed >> 32)
 *   counter = (i mod 2^32, i >> 32, series, (day << 8) | (domain << 4) | block)
 * theta: day 0, blocks 0 and 1 give 8 words w; u = (w >> 8) 2^-24;
 *   theta_k = fl32(fl32(hi_k - lo_k) * u_k + lo_k) with one rounding (fmaf).
 * noise on day t >= 1: block 0 gives 4 words; six 21-bit fields
 *   f0..f3 = w0..w3 >> 11, f4 = (w0 & 0x7ff) << 10 | (w1 & 0x3ff),
 *   f5 = (w2 & 0x7ff) << 10 | (w3 & 0x3ff); u = (f + 1/2) 2^-21;
 *   Box-Muller pairs (u0,u1), (u2,u3), (u4,u5) with r = sqrt(-2 ln u_even):
 *   z1 = r0 cos(2 pi u1), z2 = r0 sin(2 pi u1), z3 = r1 cos(2 pi u3),
 *   z4 = r1 sin(2 pi u3), z5 = r2 cos(2 pi u5); z_k drives transition k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                       */
/* ------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

static void stream_words(uint64_t seed, uint32_t domain, uint32_t series,
                         uint64_t sample, uint32_t day, uint32_t block, uint32_t w[4])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)sample, (uint32_t)(sample >> 32), series,
                             (day << 8) | (domain << 4) | block};
    philox4x32_10(ctr, key, w);
}

ORACLE_API void oracle_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

ORACLE_API void oracle_stream_words(uint64_t seed, uint32_t domain, uint32_t series,
                                    uint64_t sample, uint32_t day, uint32_t block, uint32_t* w)
{
    stream_words(seed, domain, series, sample, day, block, w);
}

/* ------------------------------------------------------------------ */
/* Prior draw, eq. (2)                                                 */
/* ------------------------------------------------------------------ */

static void prior_theta(const float lo[8], const float hi[8], uint64_t seed, uint32_t domain,
                        uint32_t series, uint64_t sample, float theta[8])
{
    uint32_t w[8];
    stream_words(seed, domain, series, sample, 0, 0, w);
    stream_words(seed, domain, series, sample, 0, 1, w + 4);
    for (int k = 0; k < 8; ++k) {
        const float u = (float)(w[k] >> 8) * 0x1p-24f; /* exact: 24-bit integer times 2^-24 */
        const float width = hi[k] - lo[k];
        theta[k] = fmaf(width, u, lo[k]);               /* single rounding of width*u + lo */
    }
}

ORACLE_API void oracle_prior(const float* lo, const float* hi, uint64_t seed, uint32_t domain,
                             uint32_t series, uint64_t first, int64_t n, float* theta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        prior_theta(lo, hi, seed, domain, series, first + (uint64_t)i, theta + 8 * i);
}

/* ------------------------------------------------------------------ */
/* Standard normals for one (sample, day): Box-Muller on 21-bit fields */
/* ------------------------------------------------------------------ */

static void day_normals(uint64_t seed, uint32_t domain, uint32_t series, uint64_t sample,
                        uint32_t day, double z[5])
{
    uint32_t w[4];
    stream_words(seed, domain, series, sample, day, 0, w);
    uint32_t f[6];
    f[0] = w[0] >> 11;
    f[1] = w[1] >> 11;
    f[2] = w[2] >> 11;
    f[3] = w[3] >> 11;
    f[4] = ((w[0] & 0x7FFu) << 10) | (w[1] & 0x3FFu);
    f[5] = ((w[2] & 0x7FFu) << 10) | (w[3] & 0x3FFu);
    double u[6];
    for (int k = 0; k < 6; ++k) u[k] = ((double)f[k] + 0.5) * 0x1p-21;
    const double two_pi = 2.0 * M_PI;
    const double r0 = sqrt(-2.0 * log(u[0]));
    const double r1 = sqrt(-2.0 * log(u[2]));
    const double r2 = sqrt(-2.0 * log(u[4]));
    z[0] = r0 * cos(two_pi * u[1]);
    z[1] = r0 * sin(two_pi * u[1]);
    z[2] = r1 * cos(two_pi * u[3]);
    z[3] = r1 * sin(two_pi * u[3]);
    z[4] = r2 * cos(two_pi * u[5]);
}

ORACLE_API void oracle_normals(uint64_t seed, uint32_t domain, uint32_t series, uint64_t sample,
                               uint32_t day, double* z)
{
    day_normals(seed, domain, series, sample, day, z);
}

/* ------------------------------------------------------------------ */
/* Model, Sec. 2.1                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t P;           /* population at the first time point */
    int64_t A0, R0, D0;  /* observed compartments at day 0 */
    int32_t T;           /* days simulated (and compared) */
    int32_t noise_mode;  /* 0: sd = s*sqrt(h); 1: sd = s*h^(1/4) */
    int32_t dist_mode;   /* 0: log1p counts; 1: raw counts */
    int32_t pad;
    double noise_scale;  /* s; 0 gives the deterministic floor map */
} oracle_model;

/* number of transitions drawn from N(h, sd^2), floored, limited to [0, avail] */
static int64_t draw_count(const oracle_model* m, double h, double z, int64_t avail)
{
    double sd;
    if (m->noise_mode == 0)
        sd = m->noise_scale * sqrt(h);
    else
        sd = m->noise_scale * sqrt(sqrt(h));
    const double x = h + sd * z;
    const double f = floor(x);
    if (!(f > 0.0)) return 0; /* negative, or NaN from a negative rate */
    if (f >= (double)avail) return avail;
    return (int64_t)f;
}

/*
 * One trajectory. theta holds the FP32 parameter values (widened exactly).
 * traj (nullable) receives (T+1) rows of (S, I, A, R, D, Ru), day 0 first.
 * obs (nullable) is [3][T] (A, R, D for days 1..T); the return value is the
 * distance over days 1..T, or 0 when obs is NULL.
 */
static double trajectory(const oracle_model* m, const float theta_f[8], uint64_t seed,
                         uint32_t domain, uint32_t series, uint64_t sample,
                         const int32_t* obs, int64_t* traj)
{
    double th[8];
    for (int k = 0; k < 8; ++k) th[k] = (double)theta_f[k];
    const double alpha0 = th[0], alpha = th[1], n_exp = th[2], beta = th[3];
    const double gamma = th[4], delta = th[5], eta = th[6], kappa = th[7];

    int64_t A = m->A0, R = m->R0, D = m->D0, Ru = 0;
    int64_t I = (int64_t)floor(kappa * (double)m->A0);
    if (I > m->P - (A + R + D)) I = m->P - (A + R + D); /* S cannot go negative */
    int64_t S = m->P - (A + R + D + I);
    const double P = (double)m->P;

    if (traj) {
        int64_t* row = traj;
        row[0] = S; row[1] = I; row[2] = A; row[3] = R; row[4] = D; row[5] = Ru;
    }
    double acc = 0.0;
    for (int t = 1; t <= m->T; ++t) {
        const double M = (double)(A + R + D);
        const double g = alpha0 + alpha / (1.0 + pow(M, n_exp));
        const double h1 = g * (double)S * (double)I / P;
        const double h2 = gamma * (double)I;
        const double h3 = beta * (double)A;
        const double h4 = delta * (double)A;
        const double h5 = beta * eta * (double)I;

        double z[5];
        day_normals(seed, domain, series, sample, (uint32_t)t, z);

        const int64_t n1 = draw_count(m, h1, z[0], S);
        const int64_t n2 = draw_count(m, h2, z[1], I);
        const int64_t n3 = draw_count(m, h3, z[2], A);
        const int64_t n4 = draw_count(m, h4, z[3], A - n3);
        const int64_t n5 = draw_count(m, h5, z[4], I - n2);

        S -= n1;
        I += n1 - n2 - n5;
        A += n2 - n3 - n4;
        R += n3;
        D += n4;
        Ru += n5;

        if (traj) {
            int64_t* row = traj + 6 * t;
            row[0] = S; row[1] = I; row[2] = A; row[3] = R; row[4] = D; row[5] = Ru;
        }
        if (obs) {
            const int64_t X[3] = {A, R, D};
            for (int c = 0; c < 3; ++c) {
                const int64_t O = obs[c * m->T + (t - 1)];
                double d;
                if (m->dist_mode == 0)
                    d = log1p((double)X[c]) - log1p((double)O);
                else
                    d = (double)X[c] - (double)O;
                acc += d * d;
            }
        }
    }
    return sqrt(acc);
}

ORACLE_API double oracle_trajectory(const oracle_model* m, const float* theta, uint64_t seed,
                                    uint32_t domain, uint32_t series, uint64_t sample,
                                    const int32_t* obs, int64_t* traj)
{
    return trajectory(m, theta, seed, domain, series, sample, obs, traj);
}

/*
 * Distances for samples first..first+n-1 of one series. theta is [n][8]
 * (FP32) or NULL, in which case each sample's theta is drawn from the prior
 * (lo, hi) with the same stream. Samples are independent; OpenMP splits them.
 */
ORACLE_API void oracle_distances(const oracle_model* m, const float* theta, const float* lo,
                                 const float* hi, uint64_t seed, uint32_t domain, uint32_t series,
                                 uint64_t first, int64_t n, const int32_t* obs, double* dist)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        float th[8];
        if (theta)
            memcpy(th, theta + 8 * i, sizeof th);
        else
            prior_theta(lo, hi, seed, domain, series, first + (uint64_t)i, th);
        dist[i] = trajectory(m, th, seed, domain, series, first + (uint64_t)i, obs, NULL);
    }
}

/* (T+1)x6 trajectories for n samples with given theta [n][8]. */
ORACLE_API void oracle_record(const oracle_model* m, const float* theta, uint64_t seed,
                              uint32_t domain, uint32_t series, uint64_t first, int64_t n,
                              int64_t* traj)
{
    const int64_t stride = 6 * (int64_t)(m->T + 1);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        trajectory(m, theta + 8 * i, seed, domain, series, first + (uint64_t)i, NULL,
                   traj + stride * i);
}

ORACLE_API int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
