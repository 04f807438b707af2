// Lower bound on the squared log1p distance still to come, shared by the
// float32 simulate kernels (one series per launch, or several).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace abc {

// ---------------------------------------------------------------------------
// Lower bound on the squared distance still to come (log1p distance only).
//
// Recovered R and dead D are cumulative: the model only ever adds to them, so
// after day t every later simulated count X_s >= X_t. Where X_t already lies
// above a later observation O_s, day s contributes at least
// (log2(1+X_t) - log2(1+O_s))^2 whatever happens in between. Summed over the
// days after t this gives F_t(a) = sum_{s>t} max(0, a - b_s)^2 with
// a = log2(1+X_t), b_s = log2(1+O_s); a sample whose running sum plus
// F_t(a_R) + F_t(a_D) already passes the exit bound cannot finish below it.
// F_t(a) grows with a and shrinks with t, so the table stores it at grid
// points a = q/2 (looked up with q rounded down) and, for each block of 2^sh
// days, at the block's last day: every lookup is a lower bound of the exact
// value. Entries are reduced by the float32 rounding the day loop can commit
// (a per-term error taken as 2^-15 in log2 units, 16 ulp of the largest log2
// count, where the hardware log2, the count's float conversion, the rounded
// observation and the subtraction together stay within a few ulp; and the
// running-sum rounding),
// so an exit taken on the bound is one the plain running sum would also have
// reached by day T: distances that are reported never change, and +INF still
// means the float32 distance ends above the exit bound.
// ---------------------------------------------------------------------------
constexpr int LB_Q = 64;          // grid a = 0, 0.5, ..., 31.5 (log2(1 + X) <= 31)
constexpr int LB_MAX_BLOCKS = 96; // time blocks per table (48 KB for R and D)

constexpr int LB_MAX_SEG = 8;      // day segments per column while building

// Builds the [2][ntb][LB_Q] table; called by every thread of the workgroup
// (it synchronises). Column (c, q) is grid point q of table c (0 = R, 1 = D);
// the days are cut into S = blockDim / 128 segments (at most 8) so that S
// threads share a column: each sums its segment, the segment sums give every
// thread the sum over the days after its segment, and each thread then walks
// its own days backwards storing the rows whose block ends there. stage holds
// b_s for R then D in float64 (2 T values, staged by the caller) followed by
// room for the [LB_MAX_SEG][2 LB_Q] segment sums.
__device__ inline void build_future_bound(double* stage, int T, int sh, int ntb, double exit2, float* tab)
{
    const double* bval = stage;
    double* segsum = stage + 2 * T;
    int S = (int)blockDim.x / (2 * LB_Q);
    S = S < 1 ? 1 : (S > LB_MAX_SEG ? LB_MAX_SEG : S);
    const int L = (T + S - 1) / S;
    const double e = 0x1p-15;                         // float32 error of one log2 term
    const double sum_err = 2.0 * T * 0x1p-24 * exit2; // running-sum rounding below the bound
    // phase 1: the sum of each segment
    for (int id = threadIdx.x; id < 2 * LB_Q * S; id += blockDim.x) {
        const int col = id % (2 * LB_Q), seg = id / (2 * LB_Q);
        const double g = 0.5 * (col % LB_Q);
        const double* b = bval + (col / LB_Q) * T;
        const int d0 = seg * L + 1, d1 = min((seg + 1) * L, T);
        double F = 0.0;
        for (int t = d1; t >= d0; --t) {
            const double x = g - b[t - 1];
            if (x > 0.0) F += x * x;
        }
        segsum[seg * 2 * LB_Q + col] = F;
    }
    __syncthreads();
    // phase 2 and 3: each segment's rows, from the sum over the later days
    for (int id = threadIdx.x; id < 2 * LB_Q * S; id += blockDim.x) {
        const int col = id % (2 * LB_Q), seg = id / (2 * LB_Q);
        const int c = col / LB_Q;
        const double g = 0.5 * (col % LB_Q);
        const double* b = bval + c * T;
        float* out = tab + c * ntb * LB_Q + (col % LB_Q);
        double F = 0.0;                                // sum over the days after t
        for (int k = S - 1; k > seg; --k) F += segsum[k * 2 * LB_Q + col];
        const int d0 = seg * L + 1, d1 = min((seg + 1) * L, T);
        const int tlo = seg == 0 ? 0 : d0;
        for (int t = d1; t >= tlo; --t) {
            const int tb = t >> sh;
            if (t == min(((tb + 1) << sh) - 1, T)) {
                double v = F - 2.0 * e * sqrt((double)T * F) - sum_err;
                v *= 1.0 - 0x1p-20;
                out[tb * LB_Q] = v > 0.0 ? (float)v : 0.0f;
            }
            if (t >= 1) {
                const double x = g - b[t - 1];
                if (x > 0.0) F += x * x;
            }
        }
    }
}

}  // namespace abc
