// Prior sampling, simulate+distance and trajectory recording kernels, and their
// C-ABI entry points (abc_sample_prior, abc_simulate_distance,
// abc_simulate_record).
//
// simulate+distance: one lane per trajectory. The observed series of the
// launch is staged once per workgroup in LDS as log1p(O) (or O for the raw
// distance), so the day loop touches no global memory at all: per sample the
// kernel reads 32 B of theta (or none when theta is drawn in-kernel) and
// writes 4 B of distance. A sample leaves the day loop as soon as its running
// squared distance passes the early-exit bound.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "model.hpp"

namespace abc {

constexpr int SIM_BLOCK = 256;

struct SimArgs {
    const float* theta;  // [n][8] or null -> prior draw
    float lo[8];
    float width[8];
    Key key;
    uint32_t domain;
    uint32_t series;
    uint64_t first;
    int64_t n;
    int32_t P, A0, R0, D0, T;
    const int32_t* obs;  // [3][T]
    float scale;
    float exit_f32;      // squared-distance early-exit bound (float path)
    double exit_f64;     // same, double path
    float* dist;
    double* dist64;
    int32_t* traj;       // record mode: [n][T+1][6]
};

__device__ __forceinline__ void load_or_draw_theta(const SimArgs& a, bool prior, int64_t k,
                                                   uint64_t i, float th[8])
{
    if (prior) {
        prior_draw(a.key, i, a.series, a.domain, a.lo, a.width, th);
    } else {
        const float4* p = reinterpret_cast<const float4*>(a.theta + 8 * k);
        const float4 x = p[0], y = p[1];
        th[0] = x.x; th[1] = x.y; th[2] = x.z; th[3] = x.w;
        th[4] = y.x; th[5] = y.y; th[6] = y.z; th[7] = y.w;
    }
}

// ---------------------------------------------------------------------------
// float32 simulate + distance
// ---------------------------------------------------------------------------
template <int NOISE, int DIST, bool KAHAN, bool PRIOR>
__global__ __launch_bounds__(SIM_BLOCK) void k_simulate_f32(SimArgs a)
{
    extern __shared__ float lds_f[];  // [3][T]: log1p(O), or O bits for DIST=1
    const int T = a.T;
    for (int q = threadIdx.x; q < 3 * T; q += blockDim.x) {
        const int32_t O = a.obs[q];
        if (DIST == 0)
            lds_f[q] = (float)log1p((double)O);
        else
            lds_f[q] = __int_as_float(O);
    }
    __syncthreads();

    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;

    float thv[8];
    load_or_draw_theta(a, PRIOR, k, i, thv);
    const Theta th = theta_from(thv);
    const RatesF r = rates_f32(th);
    State s = init_state(th.ka, a.P, a.A0, a.R0, a.D0);
    const float invP = 1.0f / (float)a.P;

    float acc = 0.0f, comp = 0.0f;
    bool exited = false;
    for (int t = 1; t <= T; ++t) {
        const uint4 w = stream_words(a.key, i, a.series, ctr_word3((uint32_t)t, a.domain, 0));
        float z[5];
        normals_f32(w, z);
        day_step_f32<NOISE>(s, r, invP, a.scale, z);
        const int32_t X[3] = {s.A, s.R, s.D};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float d;
            if (DIST == 0)
                d = log1p_count_f32(X[c]) - lds_f[c * T + t - 1];
            else
                d = (float)(X[c] - __float_as_int(lds_f[c * T + t - 1]));
            if (KAHAN) {
                const float y = d * d - comp;
                const float tt = acc + y;
                comp = (tt - acc) - y;
                acc = tt;
            } else {
                acc = fmaf(d, d, acc);
            }
        }
        if (acc > a.exit_f32) {
            exited = true;
            break;
        }
    }
    const float dd = exited ? INFINITY : sqrtf(acc);
    a.dist[k] = dd;
    if (a.dist64) a.dist64[k] = (double)dd;
}

// ---------------------------------------------------------------------------
// float64 simulate + distance (precision study, recheck of borderline samples)
// ---------------------------------------------------------------------------
template <int NOISE, int DIST, bool PRIOR>
__global__ __launch_bounds__(SIM_BLOCK) void k_simulate_f64(SimArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ double lds_d[];  // [3][T]: log1p(O) or O
    const int T = a.T;
    for (int q = threadIdx.x; q < 3 * T; q += blockDim.x) {
        const int32_t O = a.obs[q];
        lds_d[q] = DIST == 0 ? log1p((double)O) : (double)O;
    }
    __syncthreads();

    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;

    float thv[8];
    load_or_draw_theta(a, PRIOR, k, i, thv);
    const Theta th = theta_from(thv);
    State s = init_state(th.ka, a.P, a.A0, a.R0, a.D0);
    const double P = (double)a.P;
    const double scale = (double)a.scale;

    double acc = 0.0;
    bool exited = false;
    for (int t = 1; t <= T; ++t) {
        const uint4 w = stream_words(a.key, i, a.series, ctr_word3((uint32_t)t, a.domain, 0));
        double z[5];
        normals_f64(w, z);
        day_step_f64<NOISE>(s, th, P, scale, z);
        const int32_t X[3] = {s.A, s.R, s.D};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double d;
            if (DIST == 0)
                d = log1p((double)X[c]) - lds_d[c * T + t - 1];
            else
                d = (double)X[c] - lds_d[c * T + t - 1];
            acc += d * d;
        }
        if (acc > a.exit_f64) {
            exited = true;
            break;
        }
    }
    const double dd = exited ? (double)INFINITY : sqrt(acc);
    a.dist[k] = (float)dd;
    if (a.dist64) a.dist64[k] = dd;
}

// ---------------------------------------------------------------------------
// trajectory recording (float32 or float64 arithmetic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_state(int32_t* row, const State& s)
{
    row[0] = s.S; row[1] = s.I; row[2] = s.A; row[3] = s.R; row[4] = s.D; row[5] = s.Ru;
}

template <int NOISE, bool F64>
__global__ __launch_bounds__(SIM_BLOCK) void k_record(SimArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;
    float thv[8];
    load_or_draw_theta(a, false, k, i, thv);
    const Theta th = theta_from(thv);
    State s = init_state(th.ka, a.P, a.A0, a.R0, a.D0);
    int32_t* out = a.traj + (int64_t)6 * (a.T + 1) * k;
    store_state(out, s);
    const RatesF r = rates_f32(th);
    const float invP = 1.0f / (float)a.P;
    for (int t = 1; t <= a.T; ++t) {
        const uint4 w = stream_words(a.key, i, a.series, ctr_word3((uint32_t)t, a.domain, 0));
        if (F64) {
            double z[5];
            normals_f64(w, z);
            day_step_f64<NOISE>(s, th, (double)a.P, (double)a.scale, z);
        } else {
            float z[5];
            normals_f32(w, z);
            day_step_f32<NOISE>(s, r, invP, a.scale, z);
        }
        store_state(out + 6 * t, s);
    }
}

// ---------------------------------------------------------------------------
// prior sampling
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SIM_BLOCK) void k_sample_prior(SimArgs a, float* theta)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    float th[8];
    prior_draw(a.key, a.first + (uint64_t)k, a.series, a.domain, a.lo, a.width, th);
    float4* p = reinterpret_cast<float4*>(theta + 8 * k);
    p[0] = make_float4(th[0], th[1], th[2], th[3]);
    p[1] = make_float4(th[4], th[5], th[6], th[7]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static abc_status fill_series(SimArgs& a, const abc_series* ser, const abc_model* m,
                              const abc_stream* st, uint64_t first, int64_t n)
{
    a.key = make_key(st->seed);
    a.domain = st->domain;
    a.series = st->series;
    a.first = first;
    a.n = n;
    a.P = (int32_t)ser->P;
    a.A0 = ser->A0;
    a.R0 = ser->R0;
    a.D0 = ser->D0;
    a.T = ser->T;
    a.obs = ser->obs;
    a.scale = m->noise_scale;
    return ABC_OK;
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + SIM_BLOCK - 1) / SIM_BLOCK); }

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <int NOISE, int DIST, bool KAHAN>
static void launch_f32(const SimArgs& a, bool prior, size_t lds, hipStream_t s)
{
    if (prior)
        hipLaunchKernelGGL((k_simulate_f32<NOISE, DIST, KAHAN, true>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
    else
        hipLaunchKernelGGL((k_simulate_f32<NOISE, DIST, KAHAN, false>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
}

template <int NOISE, int DIST>
static void launch_f64(const SimArgs& a, bool prior, size_t lds, hipStream_t s)
{
    if (prior)
        hipLaunchKernelGGL((k_simulate_f64<NOISE, DIST, true>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
    else
        hipLaunchKernelGGL((k_simulate_f64<NOISE, DIST, false>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_sample_prior(const abc_prior* prior, const abc_stream* st,
                                       uint64_t first, int64_t n, float* theta, void* stream)
{
    SimArgs a{};
    abc_status rc = prior_lo_width(prior, a.lo, a.width);
    if (rc) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n = %lld < 0", (long long)n);
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(theta != nullptr && aligned16(theta), "theta must be a 16-byte aligned device pointer");
    a.key = make_key(st->seed);
    a.domain = st->domain;
    a.series = st->series;
    a.first = first;
    a.n = n;
    hipLaunchKernelGGL(k_sample_prior, dim3(grid_for(n)), dim3(SIM_BLOCK), 0, as_stream(stream),
                       a, theta);
    return check_launch("k_sample_prior");
}

extern "C" abc_status abc_simulate_distance(const abc_series* ser, const abc_model* model,
                                            const abc_stream* st, const float* theta,
                                            const abc_prior* prior, uint64_t first, int64_t n,
                                            float eps_exit, float* dist, double* dist64,
                                            void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n = %lld < 0", (long long)n);
    ABC_REQUIRE(!(eps_exit < 0.0f) && !isnan(eps_exit), "eps_exit must be >= 0 (or +INF)");
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(dist != nullptr, "dist is NULL");
    SimArgs a{};
    const bool use_prior = theta == nullptr;
    if (use_prior) {
        if ((rc = prior_lo_width(prior, a.lo, a.width))) return rc;
    } else {
        ABC_REQUIRE(aligned16(theta), "theta must be 16-byte aligned");
    }
    fill_series(a, ser, model, st, first, n);
    a.theta = theta;
    a.dist = dist;
    a.dist64 = dist64;
    // Early-exit bounds with a relative margin that keeps every exited sample
    // strictly above eps_exit after the final square root and rounding.
    const double e2 = (double)eps_exit * (double)eps_exit;
    a.exit_f32 = isinf(eps_exit) ? INFINITY : (float)(e2 * (1.0 + 0x1p-18));
    a.exit_f64 = isinf(eps_exit) ? (double)INFINITY : e2 * (1.0 + 1e-12);

    const hipStream_t s = as_stream(stream);
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const int distm = (model->flags & ABC_DIST_RAW) ? 1 : 0;
    if (model->flags & ABC_FP64) {
        const size_t lds = sizeof(double) * 3 * (size_t)a.T;
        if (noise == 0 && distm == 0) launch_f64<0, 0>(a, use_prior, lds, s);
        else if (noise == 0 && distm == 1) launch_f64<0, 1>(a, use_prior, lds, s);
        else if (noise == 1 && distm == 0) launch_f64<1, 0>(a, use_prior, lds, s);
        else launch_f64<1, 1>(a, use_prior, lds, s);
        return check_launch("k_simulate_f64");
    }
    const size_t lds = sizeof(float) * 3 * (size_t)a.T;
    const bool kahan = (model->flags & ABC_KAHAN) != 0;
    if (kahan) {
        if (noise == 0 && distm == 0) launch_f32<0, 0, true>(a, use_prior, lds, s);
        else if (noise == 0 && distm == 1) launch_f32<0, 1, true>(a, use_prior, lds, s);
        else if (noise == 1 && distm == 0) launch_f32<1, 0, true>(a, use_prior, lds, s);
        else launch_f32<1, 1, true>(a, use_prior, lds, s);
    } else {
        if (noise == 0 && distm == 0) launch_f32<0, 0, false>(a, use_prior, lds, s);
        else if (noise == 0 && distm == 1) launch_f32<0, 1, false>(a, use_prior, lds, s);
        else if (noise == 1 && distm == 0) launch_f32<1, 0, false>(a, use_prior, lds, s);
        else launch_f32<1, 1, false>(a, use_prior, lds, s);
    }
    return check_launch("k_simulate_f32");
}

extern "C" abc_status abc_simulate_record(const abc_series* ser, const abc_model* model,
                                          const abc_stream* st, const float* theta,
                                          uint64_t first, int64_t n, int32_t* traj, void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, false))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n = %lld < 0", (long long)n);
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(theta != nullptr && aligned16(theta), "theta must be a 16-byte aligned device pointer");
    ABC_REQUIRE(traj != nullptr, "traj is NULL");
    SimArgs a{};
    fill_series(a, ser, model, st, first, n);
    a.theta = theta;
    a.traj = traj;
    const hipStream_t s = as_stream(stream);
    const bool f64 = (model->flags & ABC_FP64) != 0;
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const dim3 g(grid_for(n)), b(SIM_BLOCK);
    if (f64) {
        if (noise) hipLaunchKernelGGL((k_record<1, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_record<0, true>), g, b, 0, s, a);
    } else {
        if (noise) hipLaunchKernelGGL((k_record<1, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_record<0, false>), g, b, 0, s, a);
    }
    return check_launch("k_record");
}
