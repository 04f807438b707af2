// Posterior mean and covariance of accepted theta in float64 (the per-country
// parameter averages of Table "t:trajectories", extended to the covariance
// and to importance weights), and its C-ABI entry point abc_posterior_moments.
//
// Deterministic: the rows are cut into fixed chunks of 2048; each chunk's
// sums (V1, V2, S1 = sum w (theta - c), S2 = sum w (theta - c)(theta - c)^T,
// 46 doubles) are reduced in a fixed shuffle/LDS tree, and one final
// workgroup adds the chunk sums in chunk order. The shift c is the first row,
// which keeps the centred sums free of cancellation. Then
//   mean = c + S1 / V1,  cov = (S2 - S1 S1^T / V1) / (V1 - V2 / V1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"

namespace abc {

constexpr int MOM_BLOCK = 256;
constexpr int MOM_CHUNK = 2048;
constexpr int MOM_NSUM = 2 + 8 + 36;

struct MomArgs {
    const float* theta;
    const float* weight;
    const int64_t* n_dev;
    int64_t n_max;
    int64_t nchunks;
    double* partial;  // [nchunks][MOM_NSUM]
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

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(MOM_BLOCK) void k_moments_partial(MomArgs a)
{
    __shared__ double red[MOM_BLOCK / 64][MOM_NSUM];
    const int64_t n = rows_used(a);
    const int64_t used_chunks = (n + MOM_CHUNK - 1) / MOM_CHUNK;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double c[8];
    if (n > 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = (double)a.theta[j];
    }
    for (int64_t ch = blockIdx.x; ch < used_chunks; ch += gridDim.x) {
        double s[MOM_NSUM];
#pragma unroll
        for (int q = 0; q < MOM_NSUM; ++q) s[q] = 0.0;
        for (int r = threadIdx.x; r < MOM_CHUNK; r += MOM_BLOCK) {
            const int64_t row = ch * MOM_CHUNK + r;
            if (row >= n) break;
            const double w = a.weight ? (double)a.weight[row] : 1.0;
            double x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = (double)a.theta[8 * row + j] - c[j];
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
            a.partial[ch * MOM_NSUM + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_moments_final(MomArgs a)
{
    __shared__ double tot[MOM_NSUM];
    const int64_t n = rows_used(a);
    const int64_t used_chunks = (n + MOM_CHUNK - 1) / MOM_CHUNK;
    if (threadIdx.x < MOM_NSUM) {
        double v = 0.0;
        for (int64_t ch = 0; ch < used_chunks; ++ch) v += a.partial[ch * MOM_NSUM + threadIdx.x];
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
    const hipStream_t s = as_stream(stream);
    MomArgs a{};
    a.theta = theta;
    a.weight = weight;
    a.n_dev = n_dev;
    a.n_max = n_max;
    a.nchunks = (n_max + MOM_CHUNK - 1) / MOM_CHUNK;
    a.mean = mean;
    a.cov = cov;
    void* scratch = nullptr;
    const size_t bytes = sizeof(double) * MOM_NSUM * (size_t)(a.nchunks > 0 ? a.nchunks : 1);
    ABC_HIP(hipMallocAsync(&scratch, bytes, s));
    a.partial = reinterpret_cast<double*>(scratch);
    abc_status rc = ABC_OK;
    if (a.nchunks > 0) {
        const unsigned grid = (unsigned)(a.nchunks < 1024 ? a.nchunks : 1024);
        hipLaunchKernelGGL(k_moments_partial, dim3(grid), dim3(MOM_BLOCK), 0, s, a);
        rc = check_launch("k_moments_partial");
    }
    if (rc == ABC_OK) {
        hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64), 0, s, a);
        rc = check_launch("k_moments_final");
    }
    hipError_t e = hipFreeAsync(scratch, s);
    if (rc == ABC_OK && e != hipSuccess) return set_error(ABC_EHIP, "hipFreeAsync: %s", hipGetErrorString(e));
    return rc;
}
