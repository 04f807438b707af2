// Posterior mean and covariance of accepted theta in float64 (the per-country
// parameter averages of Table "t:trajectories", extended to the covariance
// and to importance weights), and its C-ABI entry point abc_posterior_moments.
//
// Deterministic: the n rows are cut into G = min(768, ceil(n / 2048))
// contiguous ranges, a function of n alone. Workgroup b sums its range (each
// thread every 256th row, in row order; theta read as two float4 per row)
// into V1, V2, S1 = sum w (theta - c), S2 = sum w (theta - c)(theta - c)^T
// (46 doubles), reduces them in a fixed shuffle/LDS tree and writes one
// partial; one final workgroup adds the G partials in eight ordered slices
// and then the slices in order. The shift
// c is the first row, which keeps the centred sums free of cancellation. Then
//   mean = c + S1 / V1,  cov = (S2 - S1 S1^T / V1) / (V1 - V2 / V1).
// Two launches whatever n is, and the partial pass streams theta once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"

namespace abc {

constexpr int MOM_BLOCK = 256;
// Most row ranges (workgroups of the partial pass): with one step of rows
// loaded ahead the pass takes 162 VGPRs, so three wavefronts fit a SIMD and
// 768 workgroups of four wavefronts are one resident round on 256 CUs. Four
// steps ahead took 202 VGPRs (two wavefronts, 512 workgroups) and moved 6-8 %
// fewer bytes per second on 1e8 rows: the third wavefront hides more latency
// than the deeper batch.
constexpr int MOM_GROUPS = 768;
constexpr int MOM_MIN_ROWS = 2048;  // fewest rows per range
constexpr int MOM_NSUM = 2 + 8 + 36;
constexpr int MOM_BATCH = 1;        // steps of rows whose loads a thread issues together

// number of row ranges for n rows (depends on n only)
__host__ __device__ inline int64_t mom_groups(int64_t n)
{
    const int64_t g = (n + MOM_MIN_ROWS - 1) / MOM_MIN_ROWS;
    return g < MOM_GROUPS ? g : MOM_GROUPS;
}

struct MomArgs {
    const float* theta;
    const float* weight;
    const int64_t* n_dev;
    int64_t n_max;
    double* partial;  // [mom_groups(n_max)][MOM_NSUM]
    double* mean;
    double* cov;
};

__device__ __forceinline__ int64_t rows_used(const MomArgs& a)
{
    int64_t n = a.n_dev ? *a.n_dev : a.n_max;
    if (n > a.n_max) n = a.n_max;
    if (n < 0) n = 0;
    return n;
}

// Orders one wavefront's LDS writes before its lanes read what other lanes
// wrote (and reads before the next writes): a wavefront-scope fence pair
// around a wave barrier, which the compiler does not move accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(MOM_BLOCK) void k_moments_partial(MomArgs a)
{
    __shared__ double red[MOM_BLOCK / 64][MOM_NSUM];
    // per wavefront: MOM_BATCH steps of 64 theta rows (128 float4) staged
    __shared__ float4 stage[MOM_BLOCK / 64][MOM_BATCH][128];
    const int64_t n = rows_used(a);
    const int64_t G = mom_groups(n);
    if ((int64_t)blockIdx.x >= G) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t R = (n + G - 1) / G;
    const int64_t r0 = (int64_t)blockIdx.x * R;
    const int64_t r1 = r0 + R < n ? r0 + R : n;
    const float4* th4 = reinterpret_cast<const float4*>(a.theta);
    double c[8];
    {
        const float4 u = th4[0], v = th4[1];
        c[0] = u.x; c[1] = u.y; c[2] = u.z; c[3] = u.w;
        c[4] = v.x; c[5] = v.y; c[6] = v.z; c[7] = v.w;
    }
    double s[MOM_NSUM];
#pragma unroll
    for (int q = 0; q < MOM_NSUM; ++q) s[q] = 0.0;
    // Thread t sums its rows r0 + t, r0 + t + 256, ... in order. Wavefront w
    // reads the 64 consecutive rows r0 + 64 w + 256 k + [0, 64) of its step k
    // as two fully coalesced 1 KiB streams (row halves side by side), stages
    // them in LDS and each lane takes its row back; MOM_BATCH steps are
    // loaded before the float64 sums of the previous batch run.
    float4 h0[MOM_BATCH], h1[MOM_BATCH];
    float wv[MOM_BATCH];
    auto load_batch = [&](int64_t k0) {
#pragma unroll
        for (int b = 0; b < MOM_BATCH; ++b) {
            const int64_t R0 = r0 + 64 * wave + MOM_BLOCK * (k0 + b);  // first row of the step
            const int64_t i0 = 2 * R0 + lane, i1 = i0 + 64;              // float4 indices
            h0[b] = i0 < 2 * r1 ? load_stream(th4 + i0) : make_float4(0.f, 0.f, 0.f, 0.f);
            h1[b] = i1 < 2 * r1 ? load_stream(th4 + i1) : make_float4(0.f, 0.f, 0.f, 0.f);
            const int64_t row = R0 + lane;
            wv[b] = row < r1 ? (a.weight ? load_stream(a.weight + row) : 1.0f) : 0.0f;
        }
    };
    const int64_t steps = (r1 - r0 + MOM_BLOCK - 1) / MOM_BLOCK;
    load_batch(0);
    for (int64_t k0 = 0; k0 < steps; k0 += MOM_BATCH) {
        float wc[MOM_BATCH];
#pragma unroll
        for (int b = 0; b < MOM_BATCH; ++b) {
            stage[wave][b][lane] = h0[b];
            stage[wave][b][64 + lane] = h1[b];
            wc[b] = wv[b];
        }
        wave_lds_sync();
        load_batch(k0 + MOM_BATCH);  // in flight during the sums below
#pragma unroll
        for (int b = 0; b < MOM_BATCH; ++b) {
            const int64_t row = r0 + 64 * wave + MOM_BLOCK * (k0 + b) + lane;
            if (row >= r1) break;
            const float4 u = stage[wave][b][2 * lane], v = stage[wave][b][2 * lane + 1];
            const double w = (double)wc[b];
            const double x[8] = {(double)u.x - c[0], (double)u.y - c[1], (double)u.z - c[2],
                                 (double)u.w - c[3], (double)v.x - c[4], (double)v.y - c[5],
                                 (double)v.z - c[6], (double)v.w - c[7]};
            s[0] += w;
            s[1] += w * w;
#pragma unroll
            for (int j = 0; j < 8; ++j) s[2 + j] += w * x[j];
            int q = 10;
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int l = j; l < 8; ++l) s[q++] += w * x[j] * x[l];
        }
        wave_lds_sync();  // the next batch overwrites the staged rows
    }
#pragma unroll
    for (int q = 0; q < MOM_NSUM; ++q) {
        const double v = wave_sum_f64(s[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < MOM_NSUM) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < MOM_BLOCK / 64; ++w) v += red[w][threadIdx.x];
        a.partial[(int64_t)blockIdx.x * MOM_NSUM + threadIdx.x] = v;
    }
}

constexpr int MOM_FINAL_SPLIT = 8;  // the final pass sums the partials in 8 ordered slices

__global__ __launch_bounds__(64 * MOM_FINAL_SPLIT) void k_moments_final(MomArgs a)
{
    __shared__ double part[MOM_FINAL_SPLIT][MOM_NSUM];
    __shared__ double tot[MOM_NSUM];
    const int64_t n = rows_used(a);
    const int64_t G = mom_groups(n);
    const int j = threadIdx.x & 63;   // which of the 46 sums
    const int g = threadIdx.x >> 6;   // which slice of the partials
    if (j < MOM_NSUM) {
        // slice g = partials [g L, (g + 1) L) in range order, loads batched
        // ahead of the ordered adds
        const int64_t L = (G + MOM_FINAL_SPLIT - 1) / MOM_FINAL_SPLIT;
        const int64_t b0 = g * L, b1 = b0 + L < G ? b0 + L : G;
        const double* p = a.partial + j;
        double v = 0.0;
        int64_t b = b0;
        for (; b + 16 <= b1; b += 16) {
            double t[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) t[k] = p[(b + k) * MOM_NSUM];
#pragma unroll
            for (int k = 0; k < 16; ++k) v += t[k];
        }
        for (; b < b1; ++b) v += p[b * MOM_NSUM];
        part[g][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < MOM_NSUM) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < MOM_FINAL_SPLIT; ++q) v += part[q][threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (n == 0) {
        for (int j = 0; j < 8; ++j) a.mean[j] = NAN;
        for (int j = 0; j < 64; ++j) a.cov[j] = NAN;
        return;
    }
    const double v1 = tot[0], v2 = tot[1];
    const double* s1 = tot + 2;
    for (int j = 0; j < 8; ++j) a.mean[j] = (double)a.theta[j] + s1[j] / v1;
    const double denom = v1 - v2 / v1;
    int q = 10;
    for (int j = 0; j < 8; ++j)
        for (int l = j; l < 8; ++l) {
            const double cj = (tot[q++] - s1[j] * s1[l] / v1) / (denom > 0.0 ? denom : NAN);
            a.cov[8 * j + l] = cj;
            a.cov[8 * l + j] = cj;
        }
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_posterior_moments(const float* theta, const float* weight,
                                            const int64_t* n_dev, int64_t n_max, double* mean,
                                            double* cov, void* stream)
{
    ABC_REQUIRE(n_max >= 0, "n_max < 0");
    ABC_REQUIRE(mean != nullptr && cov != nullptr, "mean/cov NULL");
    ABC_REQUIRE(n_max == 0 || theta != nullptr, "theta is NULL");
    ABC_REQUIRE((reinterpret_cast<uintptr_t>(theta) & 15u) == 0, "theta must be 16-byte aligned");
    const hipStream_t s = as_stream(stream);
    MomArgs a{};
    a.theta = theta;
    a.weight = weight;
    a.n_dev = n_dev;
    a.n_max = n_max;
    a.mean = mean;
    a.cov = cov;
    const int64_t groups = mom_groups(n_max);  // enough for any device count <= n_max
    void* scratch = nullptr;
    const size_t bytes = sizeof(double) * MOM_NSUM * (size_t)(groups > 0 ? groups : 1);
    abc_status rc = stream_scratch(s, bytes, &scratch);
    if (rc) return rc;
    a.partial = reinterpret_cast<double*>(scratch);
    if (groups > 0) {
        hipLaunchKernelGGL(k_moments_partial, dim3((unsigned)groups), dim3(MOM_BLOCK), 0, s, a);
        rc = check_launch("k_moments_partial");
    }
    if (rc == ABC_OK) {
        hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64 * MOM_FINAL_SPLIT), 0, s, a);
        rc = check_launch("k_moments_final");
    }
    return rc;
}
