// Posterior-predictive bands (Sec. 5: 120-day projections from accepted
// samples with the 5th-95th percentile band): per day and compartment, the
// requested quantiles of n recorded trajectories, and its C-ABI entry point
// abc_trajectory_bands. One workgroup per (day, compartment): the n values
// are sorted in LDS (bitonic) and each quantile interpolates linearly between
// order statistics h = (n - 1) q in float64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace abc {

constexpr int BANDS_MAX_N = 8192;
constexpr int BANDS_MAX_Q = 16;

struct BandArgs {
    const int32_t* traj;  // [n][T+1][6]
    int64_t n;
    int32_t T;
    int32_t nq;
    double q[BANDS_MAX_Q];
    float* out;           // [nq][T+1][6]
};

__global__ __launch_bounds__(256) void k_bands(BandArgs a)
{
    __shared__ int32_t v[BANDS_MAX_N];
    const int day = blockIdx.x, c = blockIdx.y;
    int npow = 1;
    while (npow < a.n) npow <<= 1;
    for (int r = threadIdx.x; r < npow; r += blockDim.x)
        v[r] = r < a.n ? a.traj[((int64_t)r * (a.T + 1) + day) * 6 + c] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= npow; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < npow; t += blockDim.x) {
                const int p = t ^ j;
                if (p > t) {
                    const bool up = (t & k) == 0;
                    const int32_t x = v[t], y = v[p];
                    if ((x > y) == up) { v[t] = y; v[p] = x; }
                }
            }
            __syncthreads();
        }
    if (threadIdx.x < a.nq) {
        const double h = (double)(a.n - 1) * a.q[threadIdx.x];
        int64_t lo = (int64_t)floor(h);
        if (lo > a.n - 1) lo = a.n - 1;
        const int64_t hi = lo + 1 < a.n ? lo + 1 : lo;
        const double t = h - (double)lo;
        const double x = (double)v[lo], y = (double)v[hi];
        a.out[((int64_t)threadIdx.x * (a.T + 1) + day) * 6 + c] = (float)(x + (y - x) * t);
    }
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_trajectory_bands(const int32_t* traj, int64_t n, int32_t T,
                                           const double* q, int32_t nq, float* out, void* stream)
{
    ABC_REQUIRE(traj && q && out, "NULL argument");
    ABC_REQUIRE(n >= 1 && n <= BANDS_MAX_N, "n must be in [1, %d]", BANDS_MAX_N);
    ABC_REQUIRE(T >= 0 && T <= ABC_T_MAX, "T out of range");
    ABC_REQUIRE(nq >= 1 && nq <= BANDS_MAX_Q, "nq must be in [1, %d]", BANDS_MAX_Q);
    BandArgs a{};
    a.traj = traj;
    a.n = n;
    a.T = T;
    a.nq = nq;
    for (int k = 0; k < nq; ++k) {
        ABC_REQUIRE(q[k] >= 0.0 && q[k] <= 1.0, "quantile %d outside [0, 1]", k);
        a.q[k] = q[k];
    }
    a.out = out;
    hipLaunchKernelGGL(k_bands, dim3(T + 1, 6), dim3(256), 0, as_stream(stream), a);
    return check_launch("k_bands");
}
