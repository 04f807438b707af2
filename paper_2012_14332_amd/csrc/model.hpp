// Device-side model of Sec. 2.1 (eqs. 3-5) and the distance of Sec. 2.2.
//
// One lane owns one trajectory: the six compartments live in VGPRs as int32
// (exact for populations below 2^31), the hazards, Gaussian draws and
// distance run in float32 (or float64 for the precision study and the
// recheck of borderline samples). Nothing of the trajectory is written to
// memory; the distance is accumulated day by day.
//
// Day t >= 1 of sample i:
//   M  = A + R + D,  g = alpha0 + alpha / (1 + M^n)                   eq. (4)
//   h  = (g S I / P, gamma I, beta A, delta A, beta eta I)            eq. (5)
//   x_k = h_k + s sd(h_k) z_k with sd = sqrt(h) (or h^(1/4) literally),
//   n_k = floor(x_k) clamped to [0, what the source still holds]: S for n1,
//   I for n2, A for n3, A - n3 for n4, I - n2 for n5 (h order), then
//   S -= n1; I += n1 - n2 - n5; A += n2 - n3 - n4; R += n3; D += n4; Ru += n5.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "philox.hpp"

namespace abc {

struct State {
    int32_t S, I, A, R, D, Ru;
};

// Per-sample theta (float32 values as drawn or supplied).
struct Theta {
    float a0, al, n, be, ga, de, et, ka;
};

__device__ __forceinline__ Theta theta_from(const float t[8])
{
    return Theta{t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7]};
}

// Prior draw (eq. 2): 8 words from blocks 0 and 1 of day 0.
__device__ __forceinline__ void prior_draw(Key key, uint64_t i, uint32_t series, uint32_t domain,
                                           const float* lo, const float* width, float th[8])
{
    const uint4 a = stream_words(key, i, series, ctr_word3(0, domain, 0));
    const uint4 b = stream_words(key, i, series, ctr_word3(0, domain, 1));
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float u = (float)(w[k] >> 8) * 0x1p-24f;  // exact
        th[k] = fmaf(width[k], u, lo[k]);
    }
}

// Day-0 state: Ru = 0, I0 = floor(kappa A0) (computed exactly in double),
// S = P - (A0 + R0 + D0 + I0); I0 is limited so that S >= 0.
__device__ __forceinline__ State init_state(float kappa, int32_t P, int32_t A0, int32_t R0,
                                            int32_t D0)
{
    State s;
    s.A = A0;
    s.R = R0;
    s.D = D0;
    s.Ru = 0;
    const double i0 = floor((double)kappa * (double)A0);
    const int32_t room = P - (A0 + R0 + D0);
    s.I = i0 >= (double)room ? room : (int32_t)i0;
    s.S = room - s.I;
    return s;
}

// The six 21-bit uniforms of one day: u = (f + 1/2) 2^-21, exact in float.
__device__ __forceinline__ void day_fields(uint4 w, uint32_t f[6])
{
    f[0] = w.x >> 11;
    f[1] = w.y >> 11;
    f[2] = w.z >> 11;
    f[3] = w.w >> 11;
    f[4] = ((w.x & 0x7FFu) << 10) | (w.y & 0x3FFu);
    f[5] = ((w.z & 0x7FFu) << 10) | (w.w & 0x3FFu);
}

// ---------------------------------------------------------------------------
// float32 path: hardware transcendentals (v_log_f32 = log2, v_exp_f32 = 2^x,
// v_sqrt_f32, v_rcp_f32, v_sin/v_cos_f32 which take revolutions).
// ---------------------------------------------------------------------------

// Final float32 distance from the squared-sum accumulator: one hardware
// square root (about 1 ulp) times the unit scale (ln 2 for the log2-unit
// log1p distance, 1 for raw counts).
__device__ __forceinline__ float finish_distance_f32(float acc, float scale)
{
    return __builtin_amdgcn_sqrtf(acc) * scale;
}

// The five noise draws of one day in Box-Muller form, kept apart: the squared
// radii scaled by the noise scale s, rr_j = -2 s^2 ln u_{2j} = c log2 u_{2j}
// with c = -2 ln(2) s^2, and the angles' cosines and sines, tr_k, so that
// s z_k = sqrt(rr_j) tr_k. A draw then takes its standard deviation and its
// radius under one square root: sd(h) s z = sqrt(h rr_j) tr_k.
struct Noise32 {
    float rr[3];
    float tr[5];
};

__device__ __forceinline__ void normals_f32(uint4 w, float c, Noise32& z)
{
    uint32_t f[6];
    day_fields(w, f);
    float u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = fmaf((float)f[k], 0x1p-21f, 0x1p-22f);  // exact
    z.rr[0] = c * __builtin_amdgcn_logf(u[0]);
    z.rr[1] = c * __builtin_amdgcn_logf(u[2]);
    z.rr[2] = c * __builtin_amdgcn_logf(u[4]);
    z.tr[0] = __builtin_amdgcn_cosf(u[1]);  // cos(2 pi u1)
    z.tr[1] = __builtin_amdgcn_sinf(u[1]);
    z.tr[2] = __builtin_amdgcn_cosf(u[3]);
    z.tr[3] = __builtin_amdgcn_sinf(u[3]);
    z.tr[4] = __builtin_amdgcn_cosf(u[5]);
}

__device__ __forceinline__ float noise_c(float scale)
{
    return -1.38629436111989061883f * scale * scale;
}

// floor(h + sd(h) s z) limited to [0, avail], with s z = sqrt(rr) tr: the
// standard deviation sqrt(h) (h^(1/4) read literally) and the radius share one
// square root. For x >= 0 the float->int conversion truncates, which is the
// floor, and the clamp at 0 absorbs negative x, so no separate floor is
// needed. The float is limited below 2^31 before the conversion and the
// integer is then limited to avail, so a float rounding of avail cannot leak
// into the count. Rates are non-negative, so h >= 0 and the root is finite.
template <int NOISE>
__device__ __forceinline__ int32_t draw_f32(float h, float rr, float tr, int32_t avail)
{
    const float v = NOISE == 1 ? __builtin_amdgcn_sqrtf(h) * rr : h * rr;
    const float x = fmaf(__builtin_amdgcn_sqrtf(v), tr, h);
    const float f = __builtin_amdgcn_fmed3f(x, 0.0f, 2147483520.0f);
    return min((int32_t)f, avail);
}

struct RatesF {
    float a0, al, n, be, ga, de, bh;  // bh = beta * eta
};

__device__ __forceinline__ RatesF rates_f32(const Theta& t)
{
    return RatesF{t.a0, t.al, t.n, t.be, t.ga, t.de, t.be * t.et};
}

template <int NOISE>
__device__ __forceinline__ void day_step_f32(State& s, const RatesF& r, float invP,
                                             const Noise32& z)
{
    const float M = (float)(s.A + s.R + s.D);
    const float pw = __builtin_amdgcn_exp2f(r.n * __builtin_amdgcn_logf(M));
    const float g = fmaf(r.al, __builtin_amdgcn_rcpf(1.0f + pw), r.a0);
    const float If = (float)s.I;
    const float Af = (float)s.A;
    const float h1 = (g * invP) * (float)s.S * If;
    const float h2 = r.ga * If;
    const float h3 = r.be * Af;
    const float h4 = r.de * Af;
    const float h5 = r.bh * If;
    const int32_t n1 = draw_f32<NOISE>(h1, z.rr[0], z.tr[0], s.S);
    const int32_t n2 = draw_f32<NOISE>(h2, z.rr[0], z.tr[1], s.I);
    const int32_t n3 = draw_f32<NOISE>(h3, z.rr[1], z.tr[2], s.A);
    const int32_t n4 = draw_f32<NOISE>(h4, z.rr[1], z.tr[3], s.A - n3);
    const int32_t n5 = draw_f32<NOISE>(h5, z.rr[2], z.tr[4], s.I - n2);
    s.S -= n1;
    s.I += n1 - n2 - n5;
    s.A += n2 - n3 - n4;
    s.R += n3;
    s.D += n4;
    s.Ru += n5;
}

// log2(1 + X) of a non-negative count; the float32 distance is accumulated
// in log2 units and scaled by ln 2 once at the end.
__device__ __forceinline__ float log2p1_count_f32(int32_t X)
{
    return __builtin_amdgcn_logf((float)(X + 1));
}

// ---------------------------------------------------------------------------
// float64 path: the same definitions evaluated in the order the oracle writes
// them (no contraction), with the device math library's log/sin/cos/pow/log1p.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void normals_f64(uint4 w, double z[5])
{
#pragma clang fp contract(off)
    uint32_t f[6];
    day_fields(w, f);
    double u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = ((double)f[k] + 0.5) * 0x1p-21;
    const double two_pi = 2.0 * 3.14159265358979323846;
    const double r0 = sqrt(-2.0 * log(u[0]));
    const double r1 = sqrt(-2.0 * log(u[2]));
    const double r2 = sqrt(-2.0 * log(u[4]));
    z[0] = r0 * cos(two_pi * u[1]);
    z[1] = r0 * sin(two_pi * u[1]);
    z[2] = r1 * cos(two_pi * u[3]);
    z[3] = r1 * sin(two_pi * u[3]);
    z[4] = r2 * cos(two_pi * u[5]);
}

template <int NOISE>
__device__ __forceinline__ int32_t draw_f64(double h, double z, int32_t avail, double scale)
{
#pragma clang fp contract(off)
    double sd = NOISE == 0 ? scale * sqrt(h) : scale * sqrt(sqrt(h));
    const double x = h + sd * z;
    const double f = floor(x);
    if (!(f > 0.0)) return 0;
    if (f >= (double)avail) return avail;
    return (int32_t)f;
}

template <int NOISE>
__device__ __forceinline__ void day_step_f64(State& s, const Theta& t, double P, double scale,
                                             const double z[5])
{
#pragma clang fp contract(off)
    const double M = (double)(s.A + s.R + s.D);
    const double g = (double)t.a0 + (double)t.al / (1.0 + pow(M, (double)t.n));
    const double h1 = g * (double)s.S * (double)s.I / P;
    const double h2 = (double)t.ga * (double)s.I;
    const double h3 = (double)t.be * (double)s.A;
    const double h4 = (double)t.de * (double)s.A;
    const double h5 = (double)t.be * (double)t.et * (double)s.I;
    const int32_t n1 = draw_f64<NOISE>(h1, z[0], s.S, scale);
    const int32_t n2 = draw_f64<NOISE>(h2, z[1], s.I, scale);
    const int32_t n3 = draw_f64<NOISE>(h3, z[2], s.A, scale);
    const int32_t n4 = draw_f64<NOISE>(h4, z[3], s.A - n3, scale);
    const int32_t n5 = draw_f64<NOISE>(h5, z[4], s.I - n2, scale);
    s.S -= n1;
    s.I += n1 - n2 - n5;
    s.A += n2 - n3 - n4;
    s.R += n3;
    s.D += n4;
    s.Ru += n5;
}

// Observed series for the float64 distance: log1p(O), or O for the raw distance.
template <int DIST>
__device__ __forceinline__ void stage_obs_f64(const int32_t* obs, int T, double* lds)
{
    for (int q = threadIdx.x; q < 3 * T; q += blockDim.x) {
        const int32_t O = obs[q];
        lds[q] = DIST == 0 ? log1p((double)O) : (double)O;
    }
}

// One trajectory in float64; returns +INF once the squared distance passes
// exit_sq.
template <int NOISE, int DIST>
__device__ inline double simulate_one_f64(const float thv[8], uint64_t i, Key key, uint32_t series,
                                   uint32_t domain, int32_t P, int32_t A0, int32_t R0, int32_t D0,
                                   int T, double scale, const double* lds, double exit_sq)
{
#pragma clang fp contract(off)
    const Theta th = theta_from(thv);
    State s = init_state(th.ka, P, A0, R0, D0);
    const double Pd = (double)P;
    double acc = 0.0;
    for (int t = 1; t <= T; ++t) {
        const uint4 w = stream_words(key, i, series, ctr_word3((uint32_t)t, domain, 0));
        double z[5];
        normals_f64(w, z);
        day_step_f64<NOISE>(s, th, Pd, scale, z);
        const int32_t X[3] = {s.A, s.R, s.D};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double d;
            if (DIST == 0)
                d = log1p((double)X[c]) - lds[c * T + t - 1];
            else
                d = (double)X[c] - lds[c * T + t - 1];
            acc += d * d;
        }
        if (acc > exit_sq) return (double)INFINITY;
    }
    return sqrt(acc);
}

// Up to ROWS_PER_WAVE_MAX float64 trajectories run by one wavefront (one
// wavefront per workgroup), ROW_WINDOW days at a time: the lanes draw the
// normals of every (row, day) pair of the window in parallel, lane r walks
// row r through the window's days, the lanes form the window's squared
// distance terms in parallel, and lane r adds its row's terms in day order
// (the order of simulate_one_f64, so each result is the same double).
// A float64 instruction occupies the SIMD for the same cycles whatever its
// lane mask, so rows walked side by side in lanes cost no more than one.
// Each row's counts and running sum stay in LDS between the phases, so no
// phase holds another's registers.
// Rows r < nr: theta rth[8 r .. 8 r + 7] and sample index rix[r], in LDS.
// Scratch in LDS: zs [nr][5 ROW_WINDOW] doubles (normals, then the distance
// terms), xs [nr][3 ROW_WINDOW] int32, rw [nr] walk states. Returns row r's
// distance on lane r < nr (other lanes return 0).
constexpr int ROWS_PER_WAVE_MAX = 8;
constexpr int ROW_WINDOW = 8;

struct RowWalk {
    State s;
    int32_t pad[2];
    double acc;
};

// The three phases of a window are separate functions: each keeps its own
// constants and temporaries, so the kernel needs the registers of the largest
// phase rather than of all three.
__device__ __attribute__((noinline)) void rows_window_normals(int nr, int nd, int t0,
                                                              const uint64_t* rix, Key key,
                                                              uint32_t series, uint32_t domain,
                                                              double* zs)
{
    constexpr int ZW = 5 * ROW_WINDOW;
    const int lane = threadIdx.x & 63;
#pragma unroll 1
    for (int p = lane; p < nr * nd; p += 64) {
        const int r = p / nd, u = p - r * nd;
        const uint4 w = stream_words(key, rix[r], series, ctr_word3((uint32_t)(t0 + u), domain, 0));
        double z[5];
        normals_f64(w, z);
#pragma unroll
        for (int k = 0; k < 5; ++k) zs[r * ZW + 5 * u + k] = z[k];
    }
}

template <int NOISE>
__device__ __attribute__((noinline)) void rows_window_walk(const float* th8, State* sp,
                                                           const double* zr, int32_t* xr, int nd,
                                                           int32_t P, double scale)
{
#pragma clang fp contract(off)
    float thv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) thv[k] = th8[k];
    const Theta th = theta_from(thv);
    State s = *sp;
#pragma unroll 1
    for (int u = 0; u < nd; ++u) {
        double z[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) z[k] = zr[5 * u + k];
        day_step_f64<NOISE>(s, th, (double)P, scale, z);
        xr[3 * u + 0] = s.A;
        xr[3 * u + 1] = s.R;
        xr[3 * u + 2] = s.D;
    }
    *sp = s;
}

template <int DIST>
__device__ __attribute__((noinline)) void rows_window_terms(int nr, int nd, int t0, int T,
                                                            const int32_t* xs, const double* lobs,
                                                            double* zs)
{
#pragma clang fp contract(off)
    constexpr int ZW = 5 * ROW_WINDOW, XW = 3 * ROW_WINDOW;
    const int lane = threadIdx.x & 63;
#pragma unroll 1
    for (int p = lane; p < nr * 3 * nd; p += 64) {
        const int r = p / (3 * nd), q = p - r * 3 * nd;
        const int u = q / 3, c = q - 3 * u;
        const int t = t0 - 1 + u;  // 0-based day
        double d;
        if (DIST == 0)
            d = log1p((double)xs[r * XW + q]) - lobs[c * T + t];
        else
            d = (double)xs[r * XW + q] - lobs[c * T + t];
        zs[r * ZW + q] = d * d;
    }
}

template <int NOISE, int DIST>
__device__ double simulate_rows_f64_wave(int nr, const float* rth, const uint64_t* rix, Key key,
                                         uint32_t series, uint32_t domain, int32_t P, int32_t A0,
                                         int32_t R0, int32_t D0, int T, double scale,
                                         const double* lobs, double* zs, int32_t* xs, RowWalk* rw)
{
#pragma clang fp contract(off)
    constexpr int ZW = 5 * ROW_WINDOW, XW = 3 * ROW_WINDOW;
    const int lane = threadIdx.x & 63;
    const bool walker = lane < nr;
    if (walker) {
        rw[lane].s = init_state(rth[8 * lane + 7], P, A0, R0, D0);
        rw[lane].acc = 0.0;
    }
    for (int t0 = 1; t0 <= T; t0 += ROW_WINDOW) {
        const int nd = T - t0 + 1 < ROW_WINDOW ? T - t0 + 1 : ROW_WINDOW;
        rows_window_normals(nr, nd, t0, rix, key, series, domain, zs);
        __syncthreads();
        if (walker)
            rows_window_walk<NOISE>(rth + 8 * lane, &rw[lane].s, zs + lane * ZW, xs + lane * XW, nd,
                                    P, scale);
        __syncthreads();
        rows_window_terms<DIST>(nr, nd, t0, T, xs, lobs, zs);
        __syncthreads();
        if (walker) {
            const double* tr = zs + lane * ZW;
            double acc = rw[lane].acc;
            for (int q = 0; q < 3 * nd; ++q) acc += tr[q];
            rw[lane].acc = acc;
        }
        __syncthreads();  // the window's scratch is reused by the next one
    }
    return walker ? sqrt(rw[lane].acc) : 0.0;
}

}  // namespace abc
