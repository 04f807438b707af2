// Learned mixture-density proposal for rejection ABC: training pairs from the
// simulator itself, a 96-256-256-136 GELU network trained with hand-written
// BF16 MFMA GEMMs (FP32 accumulation) and Adam, and a defensive-mixture
// proposal sampler with importance weights. Not part of the paper, whose
// proposal is the prior (eq. 2); the prior stays both the fallback and the
// reference for the learned posterior.
//
// Network: x (96 = log1p A, R, D at 32 evenly spaced days, standardised per
// feature) -> z1 = x W1 + b1, h1 = gelu(z1) -> z2 = h1 W2 + b2, h2 = gelu(z2)
// -> out = h2 W3 + b3 = (8 logits, 8x8 means, 8x8 log sd clamped to [-7, 3])
// of a diagonal Gaussian mixture over theta standardised by the prior's mean
// and sd. Loss: mean negative log-likelihood. Parameters are float32 master
// copies [W1 96x256 | b1 | W2 256x256 | b2 | W3 256x136 | b3]; the GEMMs read
// bfloat16 copies refreshed by the Adam kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"
#include "model.hpp"
#include "proposal.hpp"

namespace abc {

constexpr int NN_IN = 96, NN_H = 256, NN_K = 8, NN_D = 8, NN_OUT = 136;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + NN_IN * NN_H, OFF_W2 = OFF_B1 + NN_H,
                  OFF_B2 = OFF_W2 + NN_H * NN_H, OFF_W3 = OFF_B2 + NN_H,
                  OFF_B3 = OFF_W3 + NN_H * NN_OUT, NN_PARAMS = OFF_B3 + NN_OUT;
constexpr float LOGSIG_LO = -7.0f, LOGSIG_HI = 3.0f;
static_assert(NN_K == MIX_K && NN_D == MIX_D && NN_OUT == MIX_OUT && LOGSIG_LO == MIX_LOGSIG_LO &&
                  LOGSIG_HI == MIX_LOGSIG_HI,
              "network output layout and proposal layout must agree");

typedef uint16_t bf16;

__device__ __forceinline__ bf16 f2bf(float x)
{
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752440f));
}

__device__ __forceinline__ float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752440f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143267794f;
}

// ----------------------------------------------------------------------------
// training pairs: theta from the prior, T and P drawn per sample, float32
// simulation, features at the 32 days d_k = 1 + rint(k (T - 1) / 31)
// ----------------------------------------------------------------------------
struct FeatArgs {
    Key key;
    uint32_t domain, series;
    uint64_t first;
    int64_t n;
    float lo[8], width[8];
    int32_t T_lo, T_hi;
    double lp_lo, lp_hi;   // log10 population range
    int32_t A0, R0, D0;
    float* features;       // [n][96] log1p counts (raw)
    float* theta;          // [n][8]
    int32_t* TP;           // [n][2] (T, P) or null
};

__device__ __forceinline__ void feature_days(int T, int d[32])
{
#pragma unroll
    for (int k = 0; k < 32; ++k) d[k] = 1 + (int)rint((double)k * (double)(T - 1) / 31.0);
}

__global__ __launch_bounds__(256) void k_mdn_features(FeatArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;
    float th[8];
    prior_draw(a.key, i, a.series, a.domain, a.lo, a.width, th);
    const uint4 w = stream_words(a.key, i, a.series, ctr_word3(0, a.domain, 2));
    const double uT = (double)(w.x >> 8) * 0x1p-24, uP = (double)(w.y >> 8) * 0x1p-24;
    int T = a.T_lo + (int)floor(uT * (double)(a.T_hi - a.T_lo + 1));
    if (T > a.T_hi) T = a.T_hi;
    double P = rint(pow(10.0, a.lp_lo + (a.lp_hi - a.lp_lo) * uP));
    if (P > 2147483647.0) P = 2147483647.0;
    const int32_t Pi = (int32_t)P;
    const Theta tt = theta_from(th);
    const RatesF r = rates_f32(tt);
    State s = init_state(tt.ka, Pi, a.A0, a.R0, a.D0);
    const float invP = 1.0f / (float)Pi;
    const float nc = noise_c(1.0f);
    const PhiloxSeries ps = philox_series(a.series, a.key);
    PhiloxDays ph;
    ph.begin(i, ps.u0, a.key);
    int days[32];
    feature_days(T, days);
    float* f = a.features + 96 * k;
    int next = 0;
    for (int t = 1; t <= T; ++t) {
        const uint4 wd = ph.day(((uint32_t)t << 8) | (a.domain << 4), ps.b1, a.key);
        Noise32 z;
        normals_f32(wd, nc, z);
        day_step_f32<0>(s, r, invP, z);
        while (next < 32 && days[next] == t) {
            f[next] = (float)log1p((double)s.A);
            f[32 + next] = (float)log1p((double)s.R);
            f[64 + next] = (float)log1p((double)s.D);
            ++next;
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) a.theta[8 * k + j] = th[j];
    if (a.TP) {
        a.TP[2 * k] = T;
        a.TP[2 * k + 1] = Pi;
    }
}

// features of an observed series [3][T]
__global__ void k_obs_features(const int32_t* obs, int T, float* out)
{
    const int q = threadIdx.x;
    if (q >= 96) return;
    int days[32];
    feature_days(T, days);
    const int c = q / 32, k = q % 32;
    out[q] = (float)log1p((double)obs[c * T + days[k] - 1]);
}

// per-feature mean and sd (float64 two-pass), one workgroup per column
__global__ __launch_bounds__(256) void k_colstats(const float* x, int64_t n, int cols, float* mean,
                                                  float* sd)
{
    __shared__ double red[4];
    const int c = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto bsum = [&](double v) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        __syncthreads();
        if (lane == 0) red[wave] = v;
        __syncthreads();
        return red[0] + red[1] + red[2] + red[3];
    };
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += (double)x[r * cols + c];
    const double mu = bsum(s) / (double)n;
    double v = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double d = (double)x[r * cols + c] - mu;
        v += d * d;
    }
    const double var = bsum(v) / (double)(n > 1 ? n - 1 : 1);
    if (threadIdx.x == 0) {
        mean[c] = (float)mu;
        sd[c] = (float)(sqrt(var) > 1e-6 ? sqrt(var) : 1e-6);
    }
}

// ----------------------------------------------------------------------------
// BF16 MFMA GEMM: C[M][N] = op(A)[M][K] op(B)[K][N], float32 accumulation.
// op(A)[m][k] = A[m lda + k] (TA = false) or A[k lda + m] (TA = true);
// op(B)[k][n] = B[k ldb + n] (TB = false) or B[n ldb + k] (TB = true).
// 64x64 workgroup tile, 4 wavefronts of 32x32, v_mfma_f32_16x16x32_bf16
// fragments, K staged through LDS in steps of 32. Epilogues:
//   EPI_STORE    C (float32), optional + bias[n]
//   EPI_GELU     Z = acc + bias -> C (float32), H = gelu(Z) as bf16
//   EPI_DGELU    acc * gelu'(Zin) -> C (float32) and H (bf16)
// grid.z splits K into equal ranges; split z writes C + z * split_stride.
// ----------------------------------------------------------------------------
constexpr int EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2;
constexpr int G_BM = 64, G_BN = 64, G_BK = 32, G_LD = G_BK + 8;

typedef float float4_t __attribute__((ext_vector_type(4)));

struct GemmArgs {
    int M, N, K;
    const bf16* A;
    int lda;
    const bf16* B;
    int ldb;
    float* C;
    int ldc;
    int64_t split_stride;
    int k_per_split;
    const float* bias;
    bf16* H;
    int ldh;
    const float* Zin;
    float* cs;  // EPI_DGELU: column-sum partials [row tiles][N], or null
};

// Staging of one K tile (BK = 32) into registers, then LDS. VEC: every
// operand row, column count and K range is a multiple of 8 elements and
// 16-byte aligned, so each thread holds one 8-element vector of A and one of B
// per K tile (one global load each); otherwise eight scalars each.
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <bool TA, bool TB, bool VEC>
struct TileRegs {
    us8 a, b;

    __device__ __forceinline__ void load(const GemmArgs& g, int tid, int m0, int n0, int k0, int kend)
    {
        const us8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (VEC) {
            if (!TA) {
                const int gm = m0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
                a = (gm < g.M && gk < kend) ? *reinterpret_cast<const us8*>(g.A + (int64_t)gm * g.lda + gk)
                                            : zero;
            } else {
                const int gm = m0 + (tid & 7) * 8, gk = k0 + (tid >> 3);
                a = (gm < g.M && gk < kend) ? *reinterpret_cast<const us8*>(g.A + (int64_t)gk * g.lda + gm)
                                            : zero;
            }
            if (TB) {
                const int gn = n0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
                b = (gn < g.N && gk < kend) ? *reinterpret_cast<const us8*>(g.B + (int64_t)gn * g.ldb + gk)
                                            : zero;
            } else {
                const int gn = n0 + (tid & 7) * 8, gk = k0 + (tid >> 3);
                b = (gn < g.N && gk < kend) ? *reinterpret_cast<const us8*>(g.B + (int64_t)gk * g.ldb + gn)
                                            : zero;
            }
        } else {
            // element e = 8 tid + q of the 64 x 32 tile, in the operand's memory order
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = 8 * tid + q;
                int mm, kk;
                if (TA) { kk = e / G_BM; mm = e % G_BM; }
                else { mm = e / G_BK; kk = e % G_BK; }
                const int gm = m0 + mm, gk = k0 + kk;
                a[q] = (gm < g.M && gk < kend) ? (TA ? g.A[(int64_t)gk * g.lda + gm] : g.A[(int64_t)gm * g.lda + gk])
                                               : (unsigned short)0;
                int nn;
                if (TB) { nn = e / G_BK; kk = e % G_BK; }
                else { kk = e / G_BN; nn = e % G_BN; }
                const int gn = n0 + nn, gk2 = k0 + kk;
                b[q] = (gn < g.N && gk2 < kend) ? (TB ? g.B[(int64_t)gn * g.ldb + gk2] : g.B[(int64_t)gk2 * g.ldb + gn])
                                                : (unsigned short)0;
            }
        }
    }

    __device__ __forceinline__ void store(bf16 (*As)[G_LD], bf16 (*Bs)[G_LD], int tid) const
    {
        if constexpr (VEC) {
            if (!TA) {
                *reinterpret_cast<us8*>(&As[tid >> 2][(tid & 3) * 8]) = a;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) As[(tid & 7) * 8 + q][tid >> 3] = a[q];
            }
            if (TB) {
                *reinterpret_cast<us8*>(&Bs[tid >> 2][(tid & 3) * 8]) = b;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) Bs[(tid & 7) * 8 + q][tid >> 3] = b[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = 8 * tid + q;
                if (TA) As[e % G_BM][e / G_BM] = a[q];
                else As[e / G_BK][e % G_BK] = a[q];
                if (TB) Bs[e / G_BK][e % G_BK] = b[q];
                else Bs[e % G_BN][e / G_BN] = b[q];
            }
        }
    }
};

// 64 x 64 workgroup tile, four wavefronts of 32 x 32, K tiles of 32 on
// gfx950's v_mfma_f32_16x16x32_bf16: lane l supplies row (l & 15) of A and
// column (l & 15) of B at k = 8 (l >> 4) + 0..7, one 16-byte LDS read per
// operand fragment, and receives C[4 (l >> 4) + r][l & 15]. The next K tile is
// loaded into registers while the current one is multiplied. With
// EPI_DGELU and cs != null, workgroup (x, y) also writes the float32 column
// sums of its 64 output rows to cs[y][n] (the bias gradient's partials).
template <bool TA, bool TB, int EPI, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g)
{
    __shared__ __align__(16) bf16 As[G_BM][G_LD];
    __shared__ __align__(16) bf16 Bs[G_BN][G_LD];  // [n][k]
    __shared__ float cs_sh[2][G_BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * G_BM, n0 = blockIdx.x * G_BN;
    const int kbeg = blockIdx.z * g.k_per_split;
    int kend = kbeg + g.k_per_split;
    if (kend > g.K) kend = g.K;
    const int wy = wave >> 1, wx = wave & 1;
    float4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

    TileRegs<TA, TB, VEC> regs;
    regs.load(g, tid, m0, n0, kbeg, kend);
    for (int k0 = kbeg; k0 < kend; k0 += G_BK) {
        regs.store(As, Bs, tid);
        __syncthreads();
        if (k0 + G_BK < kend) regs.load(g, tid, m0, n0, k0 + G_BK, kend);  // next tile in flight
        const int kq = 8 * (lane >> 4);
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(&As[wy * 32 + i * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wx * 32 + j * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float* C = g.C + (int64_t)blockIdx.z * g.split_stride;
    float csum[2] = {0.0f, 0.0f};  // this lane's column sums (j = 0, 1) over its rows
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wy * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wx * 32 + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_STORE) {
                    if (g.bias) v += g.bias[n];
                    C[(int64_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_GELU) {
                    v += g.bias[n];
                    C[(int64_t)m * g.ldc + n] = v;
                    g.H[(int64_t)m * g.ldh + n] = f2bf(gelu_f(v));
                } else {
                    v *= gelu_grad_f(g.Zin[(int64_t)m * g.ldc + n]);
                    C[(int64_t)m * g.ldc + n] = v;
                    g.H[(int64_t)m * g.ldh + n] = f2bf(v);
                    csum[j] += v;
                }
            }
    if (EPI == EPI_DGELU && g.cs) {
        // rows of the lane groups l >> 4 (fixed order), then the two wy halves
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float v = csum[j];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            csum[j] = v;
        }
        if (lane < 16) {
            cs_sh[wy][wx * 32 + lane] = csum[0];
            cs_sh[wy][wx * 32 + 16 + lane] = csum[1];
        }
        __syncthreads();
        if (tid < G_BN && n0 + tid < g.N)
            g.cs[(int64_t)blockIdx.y * g.N + n0 + tid] = cs_sh[0][tid] + cs_sh[1][tid];
    }
}

// ----------------------------------------------------------------------------
// batch assembly: rows perm(j) = (a_e j + c_e) mod n of the epoch's affine
// permutation, features standardised to bf16, theta standardised (float)
// ----------------------------------------------------------------------------
struct GatherArgs {
    const float* features;   // [n][96]
    const float* theta;      // [n][8]
    int64_t n;
    int batch;
    int steps_per_epoch;
    const int64_t* perm_ab;  // [epochs][2]
    const int32_t* step;     // device step counter (null: rows 0..batch-1 in order)
    const float* fmean;
    const float* fsd;
    float tc[8], ts[8];
    bf16* X;                 // [batch][96]
    float* T;                // [batch][8]
};

__global__ void k_gather(GatherArgs a)
{
    const int b = blockIdx.x;
    int64_t row = b;
    if (a.step) {
        const int st = *a.step;
        const int e = st / a.steps_per_epoch;
        const int64_t j = (int64_t)(st % a.steps_per_epoch) * a.batch + b;
        const int64_t pa = a.perm_ab[2 * e], pc = a.perm_ab[2 * e + 1];
        row = (pa * j + pc) % a.n;  // pa, j < n < 2^31: no overflow
    }
    for (int q = threadIdx.x; q < 96; q += blockDim.x)
        a.X[(int64_t)b * 96 + q] = f2bf((a.features[row * 96 + q] - a.fmean[q]) / a.fsd[q]);
    if (a.theta && threadIdx.x < 8)
        a.T[(int64_t)b * 8 + threadIdx.x] = (a.theta[row * 8 + threadIdx.x] - a.tc[threadIdx.x]) / a.ts[threadIdx.x];
}

// ----------------------------------------------------------------------------
// mixture negative log-likelihood and its gradient w.r.t. the 136 outputs
// (divided by the batch size); loss_acc[0] += sum of NLL / batch
// ----------------------------------------------------------------------------
// One workgroup of four wavefronts per LOSS_ROWS rows, a wavefront per row at
// a time; cs != null: the workgroup also writes the float32 column sums of
// its rows' gradient, cs[blockIdx][136] (the output bias's gradient partials).
constexpr int LOSS_ROWS = 64;

__global__ __launch_bounds__(256) void k_mdn_loss(const float* out, const float* T, int n,
                                                  float* dout, bf16* dout_b, float* loss_acc,
                                                  float* cs)
{
    // lane = k NN_D + j holds component k, dimension j
    static_assert(NN_K * NN_D == 64, "one lane per (component, dimension)");
    __shared__ float red[4];
    __shared__ float csh[4][NN_OUT];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k = lane / NN_D, j = lane % NN_D;
    const float inv_n = 1.0f / (float)n;
    float nll_sum = 0.0f, c_mu = 0.0f, c_ls = 0.0f, c_k = 0.0f;
    for (int q = 0; q < LOSS_ROWS / 4; ++q) {
        const int r = blockIdx.x * LOSS_ROWS + wv * (LOSS_ROWS / 4) + q;
        if (r >= n) break;  // uniform over the wavefront
        const float* o = out + (int64_t)r * NN_OUT;
        float* g = dout + (int64_t)r * NN_OUT;
        bf16* gb = dout_b + (int64_t)r * NN_OUT;
        // log-softmax of the mixture logits (every lane, same values)
        float lmax = -INFINITY;
#pragma unroll
        for (int c = 0; c < NN_K; ++c) lmax = fmaxf(lmax, o[c]);
        float se = 0.0f;
#pragma unroll
        for (int c = 0; c < NN_K; ++c) se += expf(o[c] - lmax);
        const float lse_logits = lmax + logf(se);
        // this lane's Gaussian factor
        const float mu = o[NN_K + lane];
        const float raw = o[NN_K + NN_K * NN_D + lane];
        const float ls = fminf(fmaxf(raw, LOGSIG_LO), LOGSIG_HI);
        const float si = expf(-ls);
        const float u = (T[(int64_t)r * NN_D + j] - mu) * si;
        float term = -0.5f * u * u - ls;
        term += __shfl_xor(term, 1, 64);
        term += __shfl_xor(term, 2, 64);
        term += __shfl_xor(term, 4, 64);
        const float logit = o[k];
        const float Lk = logit - lse_logits - 0.5f * NN_D * 1.83787706640934548356f + term;
        // log-sum-exp over the components (the 8 lane groups)
        float Lmax = Lk;
        Lmax = fmaxf(Lmax, __shfl_xor(Lmax, 8, 64));
        Lmax = fmaxf(Lmax, __shfl_xor(Lmax, 16, 64));
        Lmax = fmaxf(Lmax, __shfl_xor(Lmax, 32, 64));
        float sr = expf(Lk - Lmax);
        sr += __shfl_xor(sr, 8, 64);
        sr += __shfl_xor(sr, 16, 64);
        sr += __shfl_xor(sr, 32, 64);
        const float lse = Lmax + logf(sr);
        nll_sum += -lse;
        const float resp = expf(Lk - lse);
        const float gmu = -resp * u * si * inv_n;
        const float gls = (raw > LOGSIG_LO && raw < LOGSIG_HI) ? -resp * (u * u - 1.0f) * inv_n : 0.0f;
        g[NN_K + lane] = gmu;
        gb[NN_K + lane] = f2bf(gmu);
        g[NN_K + NN_K * NN_D + lane] = gls;
        gb[NN_K + NN_K * NN_D + lane] = f2bf(gls);
        c_mu += gmu;
        c_ls += gls;
        if (j == 0) {
            const float gk = (expf(logit - lse_logits) - resp) * inv_n;
            g[k] = gk;
            gb[k] = f2bf(gk);
            c_k += gk;
        }
    }
    if (lane == 0) red[wv] = nll_sum;
    if (cs) {
        csh[wv][NN_K + lane] = c_mu;
        csh[wv][NN_K + NN_K * NN_D + lane] = c_ls;
        if (j == 0) csh[wv][k] = c_k;
    }
    __syncthreads();
    // one atomic per workgroup for the logged loss (its value only)
    if (threadIdx.x == 0 && loss_acc) atomicAdd(loss_acc, (red[0] + red[1] + red[2] + red[3]) / (float)n);
    if (cs && threadIdx.x < NN_OUT) {
        const int c = threadIdx.x;
        cs[(int64_t)blockIdx.x * NN_OUT + c] = ((csh[0][c] + csh[1][c]) + csh[2][c]) + csh[3][c];
    }
}

// ----------------------------------------------------------------------------
// Adam (Kingma & Ba) on the float32 master parameters, then the bf16 copies
// of the weights; the step counter advances after every update
// ----------------------------------------------------------------------------
// The gradient of every parameter from its partials, added in fixed order:
// a weight entry from the split-K partials of its layer's product (split
// order), a bias entry from the column-sum partials of its layer (row-block
// order). With adam, the same thread then applies Adam (Kingma & Ba) to the
// float32 master parameter and refreshes its bf16 copy; the step counter
// advances afterwards (k_step_inc).
struct FinishArgs {
    const float* part1;   // [splits][96][256]
    const float* part2;   // [splits][256][256]
    const float* part3;   // [splits][256][136]
    int splits;
    const float* cs1;     // [row tiles][256]
    const float* cs2;     // [row tiles][256]
    const float* cs3;     // [loss blocks][136]
    int tiles, lblocks;
    float* g;
    int adam;
    float* p;
    float* m;
    float* v;
    bf16* pb;
    const int32_t* step;
    float lr, b1, b2, eps;
};

__global__ void k_grad_finish(FinishArgs a)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NN_PARAMS) return;
    const float* src;
    int64_t stride;
    int cnt;
    if (e < OFF_B1) { src = a.part1 + e; stride = (int64_t)NN_IN * NN_H; cnt = a.splits; }
    else if (e < OFF_W2) { src = a.cs1 + (e - OFF_B1); stride = NN_H; cnt = a.tiles; }
    else if (e < OFF_B2) { src = a.part2 + (e - OFF_W2); stride = (int64_t)NN_H * NN_H; cnt = a.splits; }
    else if (e < OFF_W3) { src = a.cs2 + (e - OFF_B2); stride = NN_H; cnt = a.tiles; }
    else if (e < OFF_B3) { src = a.part3 + (e - OFF_W3); stride = (int64_t)NN_H * NN_OUT; cnt = a.splits; }
    else { src = a.cs3 + (e - OFF_B3); stride = NN_OUT; cnt = a.lblocks; }
    // in order, loads issued eight ahead of the adds
    float gsum = 0.0f;
    int z = 0;
    for (; z + 8 <= cnt; z += 8) {
        float t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = src[(int64_t)(z + q) * stride];
#pragma unroll
        for (int q = 0; q < 8; ++q) gsum += t[q];
    }
    for (; z < cnt; ++z) gsum += src[(int64_t)z * stride];
    a.g[e] = gsum;
    if (!a.adam) return;
    const int st = *a.step + 1;
    const float m = a.b1 * a.m[e] + (1.0f - a.b1) * gsum;
    const float v = a.b2 * a.v[e] + (1.0f - a.b2) * gsum * gsum;
    a.m[e] = m;
    a.v[e] = v;
    const float mh = m / (1.0f - powf(a.b1, (float)st));
    const float vh = v / (1.0f - powf(a.b2, (float)st));
    const float p = a.p[e] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.p[e] = p;
    a.pb[e] = f2bf(p);
}

__global__ void k_step_inc(int32_t* step, float* loss_log, const float* loss_acc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (loss_log) loss_log[*step] = *loss_acc;
        *step += 1;
    }
}

__global__ void k_zero_f32(float* p, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.0f;
}

__global__ void k_to_bf16(const float* p, int64_t n, bf16* out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = f2bf(p[e]);
}

// initialisation (domain 3 stream): W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0
__global__ void k_mdn_init(float* p, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NN_PARAMS) return;
    int fan_in = 0;
    if (e < OFF_B1) fan_in = NN_IN;
    else if (e >= OFF_W2 && e < OFF_B2) fan_in = NN_H;
    else if (e >= OFF_W3 && e < OFF_B3) fan_in = NN_H;
    float v = 0.0f;
    if (fan_in) {
        const uint4 w = stream_words(make_key(seed), (uint64_t)e, 0, ctr_word3(0, 3, 0));
        const float u = (float)(w.x >> 8) * 0x1p-24f;
        v = (2.0f * u - 1.0f) * rsqrtf((float)fan_in);
    }
    p[e] = v;
}

// ----------------------------------------------------------------------------
// defensive-mixture proposal: with probability lambda a prior draw, else a
// draw from the network's mixture for one series, mapped back to theta units;
// draws outside the prior box are redrawn (attempt a uses day a + 1 of the
// proposal stream). weight = prior density / q, q = (1 - lambda) q_mix +
// lambda prior (q_mix carries the Jacobian of the standardisation). The
// truncation's normalising constant cancels under self-normalised weights.
// ----------------------------------------------------------------------------
struct SampleArgs {
    const float* mix;     // [136] network output for the series
    ProposalBox prop;
    Key key;
    uint32_t domain, series;
    uint64_t first;
    int64_t n;
    float* theta;         // [n][8]
    float* weight;        // [n]
};

__global__ __launch_bounds__(256) void k_mdn_sample(SampleArgs a)
{
    __shared__ float o[NN_OUT];
    __shared__ MixTable tab;
    for (int q = threadIdx.x; q < NN_OUT; q += blockDim.x) o[q] = a.mix[q];
    __syncthreads();
    if (threadIdx.x < MIX_K * MIX_D) mix_table_entry(o, a.prop, threadIdx.x / MIX_D, threadIdx.x % MIX_D, tab);
    __syncthreads();
    if (threadIdx.x == 0) mix_table_finish(o, tab);
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    float th[8];
    const float w = proposal_draw(tab, a.prop, a.key, a.first + (uint64_t)k, a.series, a.domain, th);
    for (int j = 0; j < 8; ++j) a.theta[8 * k + j] = th[j];
    a.weight[k] = w;
}

// K range per split for the weight-gradient products (reduction over the
// batch): 128 rows per split once K >= 512, else no split.
static int k_per_split_for(int K) { return K >= 512 ? 128 : ((K + G_BK - 1) / G_BK) * G_BK; }
static int splits_for(int K) { const int kps = k_per_split_for(K); return (K + kps - 1) / kps; }

// kps = K range per split (0: the whole K in one split)
template <bool TA, bool TB, int EPI>
static void gemm(const GemmArgs& g0, int kps, hipStream_t s)
{
    GemmArgs g = g0;
    g.k_per_split = kps > 0 ? kps : ((g.K + G_BK - 1) / G_BK) * G_BK;
    const int splits = (g.K + g.k_per_split - 1) / g.k_per_split;
    g.split_stride = (int64_t)g.M * g.N;
    const dim3 grid((g.N + G_BN - 1) / G_BN, (g.M + G_BM - 1) / G_BM, splits);
    const bool vec = g.M % 8 == 0 && g.N % 8 == 0 && g.K % 8 == 0 && g.lda % 8 == 0 &&
                     g.ldb % 8 == 0 && g.k_per_split % 8 == 0 &&
                     (reinterpret_cast<uintptr_t>(g.A) & 15u) == 0 &&
                     (reinterpret_cast<uintptr_t>(g.B) & 15u) == 0;
    if (vec)
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, true>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, false>), grid, dim3(256), 0, s, g);
}

}  // namespace abc

using namespace abc;

struct abc_mdn {
    float* p = nullptr;
    bf16* pb = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* g = nullptr;
    float* fmean = nullptr;
    float* fsd = nullptr;
    int32_t* step = nullptr;
    float* loss_acc = nullptr;
    float lo[8], hi[8], tc[8], ts[8];
    int ws = 0;  // workspace rows
    bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *dOUTb = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    float *T = nullptr, *Z1 = nullptr, *Z2 = nullptr, *OUT = nullptr, *dOUT = nullptr,
          *dZ2 = nullptr, *dZ1 = nullptr;
    // split-K partials of the three weight gradients, column-sum partials of
    // the three bias gradients
    float *part1 = nullptr, *part2 = nullptr, *part3 = nullptr, *cs1 = nullptr, *cs2 = nullptr,
          *cs3 = nullptr;
    int64_t* perm = nullptr;
};

namespace {

void free_ws(abc_mdn* n)
{
    void* ptrs[] = {n->X, n->H1, n->H2, n->dOUTb, n->dZ2b, n->dZ1b, n->T, n->Z1, n->Z2,
                    n->OUT, n->dOUT, n->dZ2, n->dZ1, n->part1, n->part2, n->part3,
                    n->cs1, n->cs2, n->cs3};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    n->X = n->H1 = n->H2 = n->dOUTb = n->dZ2b = n->dZ1b = nullptr;
    n->T = n->Z1 = n->Z2 = n->OUT = n->dOUT = n->dZ2 = n->dZ1 = nullptr;
    n->part1 = n->part2 = n->part3 = n->cs1 = n->cs2 = n->cs3 = nullptr;
    n->ws = 0;
}

abc_status ensure_ws(abc_mdn* n, int rows)
{
    if (rows <= n->ws) return ABC_OK;
    free_ws(n);
    const size_t r = (size_t)rows;
    const int splits = splits_for(rows);
#define ALLOC(ptr, bytes) ABC_HIP(hipMalloc((void**)&(ptr), (bytes)))
    ALLOC(n->X, r * NN_IN * sizeof(bf16));
    ALLOC(n->T, r * NN_D * sizeof(float));
    ALLOC(n->Z1, r * NN_H * sizeof(float));
    ALLOC(n->H1, r * NN_H * sizeof(bf16));
    ALLOC(n->Z2, r * NN_H * sizeof(float));
    ALLOC(n->H2, r * NN_H * sizeof(bf16));
    ALLOC(n->OUT, r * NN_OUT * sizeof(float));
    ALLOC(n->dOUT, r * NN_OUT * sizeof(float));
    ALLOC(n->dOUTb, r * NN_OUT * sizeof(bf16));
    ALLOC(n->dZ2, r * NN_H * sizeof(float));
    ALLOC(n->dZ2b, r * NN_H * sizeof(bf16));
    ALLOC(n->dZ1, r * NN_H * sizeof(float));
    ALLOC(n->dZ1b, r * NN_H * sizeof(bf16));
    ALLOC(n->part1, (size_t)splits * NN_IN * NN_H * sizeof(float));
    ALLOC(n->part2, (size_t)splits * NN_H * NN_H * sizeof(float));
    ALLOC(n->part3, (size_t)splits * NN_H * NN_OUT * sizeof(float));
    ALLOC(n->cs1, (size_t)((rows + G_BM - 1) / G_BM) * NN_H * sizeof(float));
    ALLOC(n->cs2, (size_t)((rows + G_BM - 1) / G_BM) * NN_H * sizeof(float));
    ALLOC(n->cs3, (size_t)((rows + LOSS_ROWS - 1) / LOSS_ROWS) * NN_OUT * sizeof(float));
#undef ALLOC
    n->ws = rows;
    return ABC_OK;
}

void launch_gather(abc_mdn* net, const float* features, const float* theta, int64_t n_rows,
                   int batch, int steps_per_epoch, const int64_t* perm, const int32_t* step,
                   hipStream_t s)
{
    GatherArgs ga{};
    ga.features = features;
    ga.theta = theta;
    ga.n = n_rows;
    ga.batch = batch;
    ga.steps_per_epoch = steps_per_epoch;
    ga.perm_ab = perm;
    ga.step = step;
    ga.fmean = net->fmean;
    ga.fsd = net->fsd;
    for (int j = 0; j < 8; ++j) { ga.tc[j] = net->tc[j]; ga.ts[j] = net->ts[j]; }
    ga.X = net->X;
    ga.T = net->T;
    hipLaunchKernelGGL(k_gather, dim3(batch), dim3(128), 0, s, ga);
}

void forward(abc_mdn* net, int n, hipStream_t s)
{
    GemmArgs g{};
    g.M = n; g.N = NN_H; g.K = NN_IN;
    g.A = net->X; g.lda = NN_IN; g.B = net->pb + OFF_W1; g.ldb = NN_H;
    g.C = net->Z1; g.ldc = NN_H; g.bias = net->p + OFF_B1; g.H = net->H1; g.ldh = NN_H;
    gemm<false, false, EPI_GELU>(g, 0, s);
    g = GemmArgs{};
    g.M = n; g.N = NN_H; g.K = NN_H;
    g.A = net->H1; g.lda = NN_H; g.B = net->pb + OFF_W2; g.ldb = NN_H;
    g.C = net->Z2; g.ldc = NN_H; g.bias = net->p + OFF_B2; g.H = net->H2; g.ldh = NN_H;
    gemm<false, false, EPI_GELU>(g, 0, s);
    g = GemmArgs{};
    g.M = n; g.N = NN_OUT; g.K = NN_H;
    g.A = net->H2; g.lda = NN_H; g.B = net->pb + OFF_W3; g.ldb = NN_OUT;
    g.C = net->OUT; g.ldc = NN_OUT; g.bias = net->p + OFF_B3;
    gemm<false, false, EPI_STORE>(g, 0, s);
}

// loss and the gradient partials of the mean NLL (forward must have run); the
// gradient itself is formed by k_grad_finish
void backward(abc_mdn* net, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mdn_loss, dim3((n + LOSS_ROWS - 1) / LOSS_ROWS), dim3(256), 0, s, net->OUT,
                       net->T, n, net->dOUT, net->dOUTb, net->loss_acc, net->cs3);
    const int kps = k_per_split_for(n);
    // dW3 = H2^T dOUT (db3: the loss kernel's column partials)
    GemmArgs g{};
    g.M = NN_H; g.N = NN_OUT; g.K = n;
    g.A = net->H2; g.lda = NN_H; g.B = net->dOUTb; g.ldb = NN_OUT;
    g.C = net->part3; g.ldc = NN_OUT;
    gemm<true, false, EPI_STORE>(g, kps, s);
    // dZ2 = (dOUT W3^T) gelu'(Z2), with the column partials of db2
    g = GemmArgs{};
    g.M = n; g.N = NN_H; g.K = NN_OUT;
    g.A = net->dOUTb; g.lda = NN_OUT; g.B = net->pb + OFF_W3; g.ldb = NN_OUT;
    g.C = net->dZ2; g.ldc = NN_H; g.Zin = net->Z2; g.H = net->dZ2b; g.ldh = NN_H; g.cs = net->cs2;
    gemm<false, true, EPI_DGELU>(g, 0, s);
    // dW2 = H1^T dZ2
    g = GemmArgs{};
    g.M = NN_H; g.N = NN_H; g.K = n;
    g.A = net->H1; g.lda = NN_H; g.B = net->dZ2b; g.ldb = NN_H;
    g.C = net->part2; g.ldc = NN_H;
    gemm<true, false, EPI_STORE>(g, kps, s);
    // dZ1 = (dZ2 W2^T) gelu'(Z1), with the column partials of db1
    g = GemmArgs{};
    g.M = n; g.N = NN_H; g.K = NN_H;
    g.A = net->dZ2b; g.lda = NN_H; g.B = net->pb + OFF_W2; g.ldb = NN_H;
    g.C = net->dZ1; g.ldc = NN_H; g.Zin = net->Z1; g.H = net->dZ1b; g.ldh = NN_H; g.cs = net->cs1;
    gemm<false, true, EPI_DGELU>(g, 0, s);
    // dW1 = X^T dZ1
    g = GemmArgs{};
    g.M = NN_IN; g.N = NN_H; g.K = n;
    g.A = net->X; g.lda = NN_IN; g.B = net->dZ1b; g.ldb = NN_H;
    g.C = net->part1; g.ldc = NN_H;
    gemm<true, false, EPI_STORE>(g, kps, s);
}

FinishArgs finish_args(abc_mdn* net, int n)
{
    FinishArgs f{};
    f.part1 = net->part1; f.part2 = net->part2; f.part3 = net->part3;
    f.splits = splits_for(n);
    f.cs1 = net->cs1; f.cs2 = net->cs2; f.cs3 = net->cs3;
    f.tiles = (n + G_BM - 1) / G_BM;
    f.lblocks = (n + LOSS_ROWS - 1) / LOSS_ROWS;
    f.g = net->g;
    return f;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" int64_t abc_mdn_param_count(void) { return NN_PARAMS; }

extern "C" abc_status abc_mdn_create(const abc_prior* prior, uint64_t init_seed, abc_mdn** out)
{
    ABC_REQUIRE(out != nullptr, "out is NULL");
    float lo[8], width[8];
    abc_status rc = prior_lo_width(prior, lo, width);
    if (rc) return rc;
    for (int j = 0; j < 8; ++j) ABC_REQUIRE(width[j] > 0.0f, "prior box %d has zero width", j);
    abc_mdn* n = new abc_mdn();
    for (int j = 0; j < 8; ++j) {
        n->lo[j] = prior->lo[j];
        n->hi[j] = prior->hi[j];
        n->tc[j] = 0.5f * (prior->lo[j] + prior->hi[j]);
        n->ts[j] = (prior->hi[j] - prior->lo[j]) / 3.46410161513775458705f;  // as proposal_standardiser
    }
    hipError_t e = hipSuccess;
    e = e ? e : hipMalloc((void**)&n->p, NN_PARAMS * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->pb, NN_PARAMS * sizeof(bf16));
    e = e ? e : hipMalloc((void**)&n->m, NN_PARAMS * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->v, NN_PARAMS * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->g, NN_PARAMS * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->fmean, NN_IN * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->fsd, NN_IN * sizeof(float));
    e = e ? e : hipMalloc((void**)&n->step, sizeof(int32_t));
    e = e ? e : hipMalloc((void**)&n->loss_acc, sizeof(float));
    if (e != hipSuccess) {
        abc_mdn_destroy(n);
        return set_error(ABC_EHIP, "abc_mdn_create: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_mdn_init, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, 0, n->p, init_seed);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, 0, n->p, NN_PARAMS, n->pb);
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, 0, n->m, NN_PARAMS);
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, 0, n->v, NN_PARAMS);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(NN_IN), 0, 0, n->fmean, NN_IN);
    std::vector<float> ones(NN_IN, 1.0f);
    e = hipMemcpy(n->fsd, ones.data(), NN_IN * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->step, 0, sizeof(int32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        abc_mdn_destroy(n);
        return set_error(ABC_EHIP, "abc_mdn_create: %s", hipGetErrorString(e));
    }
    *out = n;
    return ABC_OK;
}

extern "C" abc_status abc_mdn_destroy(abc_mdn* n)
{
    if (!n) return ABC_OK;
    free_ws(n);
    void* ptrs[] = {n->p, n->pb, n->m, n->v, n->g, n->fmean, n->fsd, n->step, n->loss_acc, n->perm};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete n;
    return ABC_OK;
}

extern "C" abc_status abc_mdn_params(abc_mdn* n, float** params, float** grads)
{
    ABC_REQUIRE(n != nullptr, "net is NULL");
    if (params) *params = n->p;
    if (grads) *grads = n->g;
    return ABC_OK;
}

extern "C" abc_status abc_mdn_sync_params(abc_mdn* n, void* stream)
{
    ABC_REQUIRE(n != nullptr, "net is NULL");
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, as_stream(stream), n->p,
                       NN_PARAMS, n->pb);
    return check_launch("k_to_bf16");
}

extern "C" abc_status abc_mdn_simulate_features(const abc_prior* prior, uint64_t seed,
                                                uint32_t domain, uint32_t series, uint64_t first,
                                                int64_t n, int32_t T_lo, int32_t T_hi,
                                                double log10P_lo, double log10P_hi, int32_t A0,
                                                float* features, float* theta, int32_t* TP,
                                                void* stream)
{
    FeatArgs a{};
    abc_status rc = prior_lo_width(prior, a.lo, a.width);
    if (rc) return rc;
    for (int k = 0; k < 8; ++k) ABC_REQUIRE(prior->lo[k] >= 0.0f, "prior lo[%d] < 0", k);
    ABC_REQUIRE(domain <= 15u, "domain > 15");
    ABC_REQUIRE(n >= 0, "n < 0");
    ABC_REQUIRE(T_lo >= 1 && T_hi >= T_lo && T_hi <= ABC_T_MAX, "need 1 <= T_lo <= T_hi <= %d", ABC_T_MAX);
    ABC_REQUIRE(log10P_lo <= log10P_hi && log10P_hi <= 9.33, "bad population range");
    ABC_REQUIRE(A0 >= 1 && pow(10.0, log10P_lo) >= 4.0 * A0, "P must exceed 4 A0");
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(features && theta, "NULL output");
    a.key = make_key(seed);
    a.domain = domain;
    a.series = series;
    a.first = first;
    a.n = n;
    a.T_lo = T_lo;
    a.T_hi = T_hi;
    a.lp_lo = log10P_lo;
    a.lp_hi = log10P_hi;
    a.A0 = A0;
    a.features = features;
    a.theta = theta;
    a.TP = TP;
    hipLaunchKernelGGL(k_mdn_features, dim3(blocks_for(n)), dim3(256), 0, as_stream(stream), a);
    return check_launch("k_mdn_features");
}

extern "C" abc_status abc_series_features(const abc_series* ser, float* out, void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    ABC_REQUIRE(out != nullptr, "out is NULL");
    hipLaunchKernelGGL(k_obs_features, dim3(1), dim3(128), 0, as_stream(stream), ser->obs, ser->T, out);
    return check_launch("k_obs_features");
}

extern "C" abc_status abc_mdn_fit_standardizer(abc_mdn* net, const float* features, int64_t n,
                                               void* stream)
{
    ABC_REQUIRE(net && features && n >= 2, "need a net and >= 2 feature rows");
    hipLaunchKernelGGL(k_colstats, dim3(NN_IN), dim3(256), 0, as_stream(stream), features, n, NN_IN,
                       net->fmean, net->fsd);
    return check_launch("k_colstats");
}

extern "C" abc_status abc_mdn_forward(abc_mdn* net, const float* features, int64_t n, float* out,
                                      void* stream)
{
    ABC_REQUIRE(net && features && out && n >= 1 && n <= (1 << 20), "bad forward arguments");
    abc_status rc = ensure_ws(net, (int)n);
    if (rc) return rc;
    const hipStream_t s = as_stream(stream);
    // rows in order; theta is not needed (zero rows keep the gather simple)
    launch_gather(net, features, nullptr, n, (int)n, 1, nullptr, nullptr, s);
    forward(net, (int)n, s);
    ABC_HIP(hipMemcpyAsync(out, net->OUT, (size_t)n * NN_OUT * sizeof(float), hipMemcpyDeviceToDevice, s));
    return check_launch("abc_mdn_forward");
}

extern "C" abc_status abc_mdn_loss_grad(abc_mdn* net, const float* features, const float* theta,
                                        int64_t n, float* loss, float* grad, void* stream)
{
    ABC_REQUIRE(net && features && theta && n >= 1 && n <= (1 << 20), "bad arguments");
    abc_status rc = ensure_ws(net, (int)n);
    if (rc) return rc;
    const hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, net->loss_acc, (int64_t)1);
    launch_gather(net, features, theta, n, (int)n, 1, nullptr, nullptr, s);
    forward(net, (int)n, s);
    backward(net, (int)n, s);
    const FinishArgs f = finish_args(net, (int)n);
    hipLaunchKernelGGL(k_grad_finish, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, f);
    if (loss) ABC_HIP(hipMemcpyAsync(loss, net->loss_acc, sizeof(float), hipMemcpyDeviceToDevice, s));
    if (grad) ABC_HIP(hipMemcpyAsync(grad, net->g, NN_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, s));
    return check_launch("abc_mdn_loss_grad");
}

extern "C" abc_status abc_mdn_train(abc_mdn* net, const float* features, const float* theta,
                                    int64_t n, int32_t epochs, int32_t batch, float lr,
                                    uint64_t shuffle_seed, float* loss_log, int64_t* steps_out,
                                    float* train_ms, void* stream)
{
    ABC_REQUIRE(net && features && theta, "NULL argument");
    ABC_REQUIRE(n >= batch && batch >= 64 && batch <= 65536 && n < (1ll << 31), "need 64 <= batch <= n < 2^31");
    ABC_REQUIRE(epochs >= 1 && epochs <= 10000, "epochs out of range");
    ABC_REQUIRE(isfinite(lr) && lr > 0.0f, "lr must be positive");
    abc_status rc = ensure_ws(net, batch);
    if (rc) return rc;
    const int spe = (int)(n / batch);  // steps per epoch (the partial batch is dropped)
    const int64_t steps = (int64_t)spe * epochs;
    // affine permutations j -> (a j + c) mod n, one per epoch
    std::vector<int64_t> ab(2 * (size_t)epochs);
    uint64_t st = shuffle_seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto next = [&]() {  // splitmix64
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto gcd = [](int64_t x, int64_t y) { while (y) { int64_t t = x % y; x = y; y = t; } return x; };
    for (int e = 0; e < epochs; ++e) {
        int64_t a = 0;
        do { a = (int64_t)(next() % (uint64_t)n); } while (a == 0 || gcd(a, n) != 1);
        ab[2 * e] = a;
        ab[2 * e + 1] = (int64_t)(next() % (uint64_t)n);
    }
    if (net->perm) (void)hipFree(net->perm);
    net->perm = nullptr;
    ABC_HIP(hipMalloc((void**)&net->perm, ab.size() * sizeof(int64_t)));
    const hipStream_t user = as_stream(stream);
    hipStream_t s;
    ABC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct SF { hipStream_t s; ~SF() { (void)hipStreamDestroy(s); } } sf{s};
    hipEvent_t ev, t0, t1;
    ABC_HIP(hipEventCreate(&ev));
    ABC_HIP(hipEventCreate(&t0));
    ABC_HIP(hipEventCreate(&t1));
    struct EF { hipEvent_t a, b, c; ~EF() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); } } ef{ev, t0, t1};
    ABC_HIP(hipEventRecord(ev, user));
    ABC_HIP(hipStreamWaitEvent(s, ev, 0));
    ABC_HIP(hipMemcpyAsync(net->perm, ab.data(), ab.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    ABC_HIP(hipMemsetAsync(net->step, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->m, NN_PARAMS);
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->v, NN_PARAMS);
    ABC_HIP(hipStreamSynchronize(s));

    // one training step, captured once and replayed
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ABC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, net->loss_acc, (int64_t)1);
    launch_gather(net, features, theta, n, batch, spe, net->perm, net->step, s);
    forward(net, batch, s);
    backward(net, batch, s);
    FinishArgs f = finish_args(net, batch);
    f.adam = 1;
    f.p = net->p; f.m = net->m; f.v = net->v; f.pb = net->pb; f.step = net->step;
    f.lr = lr; f.b1 = 0.9f; f.b2 = 0.999f; f.eps = 1e-8f;
    hipLaunchKernelGGL(k_grad_finish, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, net->step, loss_log, net->loss_acc);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (ce != hipSuccess) return set_error(ABC_EHIP, "training graph capture: %s", hipGetErrorString(ce));
    struct GF { hipGraph_t g; hipGraphExec_t e; ~GF() { if (e) (void)hipGraphExecDestroy(e); if (g) (void)hipGraphDestroy(g); } } gf{graph, nullptr};
    ABC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    gf.e = exec;
    ABC_HIP(hipEventRecord(t0, s));
    for (int64_t k = 0; k < steps; ++k) ABC_HIP(hipGraphLaunch(exec, s));
    ABC_HIP(hipEventRecord(t1, s));
    ABC_HIP(hipEventSynchronize(t1));
    float ms = 0.0f;
    ABC_HIP(hipEventElapsedTime(&ms, t0, t1));
    if (train_ms) *train_ms = ms;
    if (steps_out) *steps_out = steps;
    ABC_HIP(hipEventRecord(ev, s));
    ABC_HIP(hipStreamWaitEvent(user, ev, 0));
    return ABC_OK;
}

extern "C" abc_status abc_mdn_sample(const abc_mdn* net, const float* mix, float lambda,
                                     float inflate, const abc_stream* st, uint64_t first,
                                     int64_t n, float* theta, float* weight, void* stream)
{
    ABC_REQUIRE(isfinite(inflate) && inflate >= 1.0f && inflate <= 100.0f, "inflate must be in [1, 100]");
    ABC_REQUIRE(net && mix, "NULL net or mixture");
    abc_status rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(lambda >= 0.0f && lambda <= 1.0f, "lambda must be in [0, 1]");
    ABC_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(theta && weight, "NULL output");
    SampleArgs a{};
    a.mix = mix;
    for (int j = 0; j < 8; ++j) {
        a.prop.lo[j] = net->lo[j]; a.prop.hi[j] = net->hi[j];
        a.prop.tc[j] = net->tc[j]; a.prop.ts[j] = net->ts[j];
    }
    a.prop.lambda = lambda;
    a.prop.log_inflate = logf(inflate);
    a.key = make_key(st->seed);
    a.domain = st->domain;
    a.series = st->series;
    a.first = first;
    a.n = n;
    a.theta = theta;
    a.weight = weight;
    hipLaunchKernelGGL(k_mdn_sample, dim3(blocks_for(n)), dim3(256), 0, as_stream(stream), a);
    return check_launch("k_mdn_sample");
}

extern "C" abc_status abc_mdn_set_params(abc_mdn* net, const float* src, void* stream)
{
    ABC_REQUIRE(net && src, "NULL argument");
    const hipStream_t s = as_stream(stream);
    ABC_HIP(hipMemcpyAsync(net->p, src, NN_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->p, NN_PARAMS, net->pb);
    return check_launch("abc_mdn_set_params");
}

extern "C" abc_status abc_mdn_get_params(const abc_mdn* net, float* dst, void* stream)
{
    ABC_REQUIRE(net && dst, "NULL argument");
    ABC_HIP(hipMemcpyAsync(dst, net->p, NN_PARAMS * sizeof(float), hipMemcpyDeviceToDevice,
                           as_stream(stream)));
    return ABC_OK;
}

extern "C" abc_status abc_mdn_get_standardizer(const abc_mdn* net, float* mean96, float* sd96,
                                               void* stream)
{
    ABC_REQUIRE(net && mean96 && sd96, "NULL argument");
    const hipStream_t s = as_stream(stream);
    ABC_HIP(hipMemcpyAsync(mean96, net->fmean, NN_IN * sizeof(float), hipMemcpyDeviceToDevice, s));
    ABC_HIP(hipMemcpyAsync(sd96, net->fsd, NN_IN * sizeof(float), hipMemcpyDeviceToDevice, s));
    return ABC_OK;
}
