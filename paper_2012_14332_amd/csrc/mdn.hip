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
// the bf16 copies: every parameter, then W3's transpose W3T [136][256]
constexpr int64_t OFF_W3T = NN_PARAMS, NN_PB = OFF_W3T + NN_H * NN_OUT;
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

// the bf16 copy of parameter e, and of its W3T entry for W3
__device__ __forceinline__ void put_bf16(bf16* pb, int64_t e, float p)
{
    const bf16 h = f2bf(p);
    pb[e] = h;
    if (e >= OFF_W3 && e < OFF_B3) {
        const int64_t q = e - OFF_W3;  // W3 [256][136]: q = k 136 + c
        pb[OFF_W3T + (q % NN_OUT) * NN_H + q / NN_OUT] = h;
    }
}

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
// batch rows: with a step counter, batch row b of training step st is dataset
// row (a_e j + c_e) mod n of epoch e's affine permutation (e = st / steps per
// epoch, j = (st mod steps per epoch) batch + b); without one, row b itself.
// Features are standardised per column, (x - mean) / sd, and theta by the
// prior's centre and sd, as they are read.
// ----------------------------------------------------------------------------
struct RowMap {
    const float* features;   // [n][96] raw features
    const float* theta;      // [n][8] or null
    int64_t n;
    int batch, steps_per_epoch;
    const int64_t* perm_ab;  // [epochs][2]
    const int32_t* step;     // device step counter, or null
    const float* fmean;
    const float* fsd;
    float tc[8], ts[8];
};

__device__ __forceinline__ int64_t map_row(const RowMap& r, int st, int b)
{
    if (!r.step) return b;
    const int e = st / r.steps_per_epoch;
    const int64_t j = (int64_t)(st % r.steps_per_epoch) * r.batch + b;
    return (r.perm_ab[2 * e] * j + r.perm_ab[2 * e + 1]) % r.n;  // a, j < n < 2^31: no overflow
}

// batch row b of step st, assembled by 128 threads (t = 0..127): standardised
// features to X [batch][96] as bf16, standardised theta to T [batch][8]
__device__ __forceinline__ void gather_row(const RowMap& rm, int st, int b, int t, bf16* X, float* T)
{
    const int64_t row = map_row(rm, st, b);
    if (t < NN_IN) X[(int64_t)b * NN_IN + t] = f2bf((rm.features[row * NN_IN + t] - rm.fmean[t]) / rm.fsd[t]);
    if (rm.theta && t < NN_D) T[(int64_t)b * NN_D + t] = (rm.theta[row * NN_D + t] - rm.tc[t]) / rm.ts[t];
}

// one workgroup of 128 threads per batch row, at the counter's step; clears
// loss_acc (nullable) for the batch's loss sum
__global__ __launch_bounds__(128) void k_gather(RowMap rm, bf16* X, float* T, float* loss_acc)
{
    if (loss_acc && blockIdx.x == 0 && threadIdx.x == 0) *loss_acc = 0.0f;
    gather_row(rm, rm.step ? *rm.step : 0, blockIdx.x, threadIdx.x, X, T);
}

// ----------------------------------------------------------------------------
// BF16 MFMA GEMM: C[M][N] = op(A)[M][K] op(B)[K][N], float32 accumulation.
// op(A)[m][k] = A[m lda + k] (TA = false) or A[k lda + m] (TA = true);
// op(B)[k][n] = B[k ldb + n] (TB = false) or B[n ldb + k] (TB = true).
// 64x64 workgroup tile, 4 wavefronts of 32x32, v_mfma_f32_16x16x32_bf16
// fragments, K staged through LDS in tiles of 64. Epilogues:
//   EPI_STORE    C (float32), optional + bias[n]
//   EPI_GELU     Z = acc + bias -> C (float32), H = gelu(Z) as bf16
//   EPI_DGELU    acc * gelu'(Zin) -> H (bf16; Zin has H's row stride)
// grid.z splits K into equal ranges; split z writes C + z * split_stride.
// ----------------------------------------------------------------------------
constexpr int EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2;
constexpr int G_BM = 64, G_BN = 64, G_BK = 64, G_LD = G_BK + 8;
constexpr int G_NT = 4, G_KMAX = G_NT * G_BK;  // K range of one workgroup: at most 4 tiles
// the products that are not split over K (forward, input gradients) reduce
// over a layer width
static_assert(NN_IN <= G_KMAX && NN_H <= G_KMAX && NN_OUT <= G_KMAX, "layer widths fit one K range");

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
    int gx, gy;          // tile grid (columns, rows); grid.z = splits
    int32_t* step_inc;   // non-null: tile (0, 0, 0) advances this counter by one
};

// Staging of one K tile (BK = 64) into registers, then LDS. Each thread holds
// G_NV = 2 eight-element vectors of A and of B per tile; vector v = tid + 256 h.
// Where K is contiguous in memory (A untransposed, B transposed) vector v is
// row v / 8, k = 8 (v % 8); where rows are contiguous it is k = v / 8, rows
// 8 (v % 8) + 0..7. VEC: every operand row, column count and K range is a
// multiple of 8 elements and 16-byte aligned, so a vector is one global load;
// otherwise it is eight scalar loads of the same elements.
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int G_NV = G_BM * G_BK / 8 / 256;

template <bool TA, bool TB, bool VEC>
struct TileRegs {
    us8 a[G_NV], b[G_NV];

    // element (r, k) of the tile for a K-contiguous (KC) or row-contiguous operand
    template <bool KC>
    __device__ static __forceinline__ void vec_pos(int v, int& r, int& k)
    {
        if (KC) { r = v >> 3; k = (v & 7) * 8; }
        else { k = v >> 3; r = (v & 7) * 8; }
    }

    template <bool KC>
    __device__ static __forceinline__ us8 load_vec(const bf16* X, int ld, int rows, int r, int k, int kend)
    {
        us8 out = {0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (VEC) {
            if (r < rows && k < kend)
                out = KC ? *reinterpret_cast<const us8*>(X + (int64_t)r * ld + k)
                         : *reinterpret_cast<const us8*>(X + (int64_t)k * ld + r);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int rr = KC ? r : r + q, kk = KC ? k + q : k;
                if (rr < rows && kk < kend)
                    out[q] = KC ? reinterpret_cast<const unsigned short*>(X)[(int64_t)rr * ld + kk]
                                : reinterpret_cast<const unsigned short*>(X)[(int64_t)kk * ld + rr];
            }
        }
        return out;
    }

    __device__ __forceinline__ void load(const GemmArgs& g, int tid, int m0, int n0, int k0, int kend)
    {
#pragma unroll
        for (int h = 0; h < G_NV; ++h) {
            const int v = tid + 256 * h;
            int r, k;
            vec_pos<!TA>(v, r, k);
            a[h] = load_vec<!TA>(g.A, g.lda, g.M, m0 + r, k0 + k, kend);
            vec_pos<TB>(v, r, k);
            b[h] = load_vec<TB>(g.B, g.ldb, g.N, n0 + r, k0 + k, kend);
        }
    }

    template <bool KC>
    __device__ static __forceinline__ void store_vec(bf16 (*S)[G_LD], int v, const us8& x)
    {
        int r, k;
        vec_pos<KC>(v, r, k);
        if (KC) {
            *reinterpret_cast<us8*>(&S[r][k]) = x;
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) reinterpret_cast<unsigned short*>(&S[r + q][k])[0] = x[q];
        }
    }

    __device__ __forceinline__ void store(bf16 (*As)[G_LD], bf16 (*Bs)[G_LD], int tid) const
    {
#pragma unroll
        for (int h = 0; h < G_NV; ++h) {
            store_vec<!TA>(As, tid + 256 * h, a[h]);
            store_vec<TB>(Bs, tid + 256 * h, b[h]);
        }
    }
};

// One 64 x 64 output tile (bx, by) of K split bz: four wavefronts of 32 x 32,
// K tiles of 64 (two MFMA steps) on gfx950's v_mfma_f32_16x16x32_bf16: lane l
// supplies row (l & 15) of A and column (l & 15) of B at k = 8 (l >> 4) + 0..7,
// one 16-byte LDS read per operand fragment, and receives C[4 (l >> 4) + r][l & 15].
// The next K tile is loaded into registers while the current one is
// multiplied. With EPI_DGELU and cs != null, tile (bx, by) also writes the
// float32 column sums of its 64 output rows to cs[by][n] (the bias gradient's
// partials).
template <bool TA, bool TB, int EPI, bool VEC>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int bx, int by, int bz, bf16 (*Ab)[G_BM][G_LD],
                                          bf16 (*Bb)[G_BN][G_LD], float (*cs_sh)[G_BN])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = by * G_BM, n0 = bx * G_BN;
    const int kbeg = bz * g.k_per_split;
    int kend = kbeg + g.k_per_split;
    if (kend > g.K) kend = g.K;
    const int wy = wave >> 1, wx = wave & 1;
    float4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

    if (g.step_inc && bx == 0 && by == 0 && bz == 0 && tid == 0) *g.step_inc += 1;
    // every K tile of the range is requested before the first is used: one
    // memory round trip per workgroup instead of one per tile
    TileRegs<TA, TB, VEC> regs[G_NT];
#pragma unroll
    for (int t = 0; t < G_NT; ++t) regs[t].load(g, tid, m0, n0, kbeg + t * G_BK, kend);
    // the epilogue's bias and (EPI_DGELU) Zin values are requested with the operands
    float bias[2] = {0.0f, 0.0f};
    if (EPI != EPI_DGELU && g.bias) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wx * 32 + j * 16 + (lane & 15);
            bias[j] = n < g.N ? g.bias[n] : 0.0f;
        }
    }
    float zin[2][2][4];
    if (EPI == EPI_DGELU) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wy * 32 + i * 16 + 4 * (lane >> 4) + r;
                    const int n = n0 + wx * 32 + j * 16 + (lane & 15);
                    zin[i][j][r] = (m < g.M && n < g.N) ? g.Zin[(int64_t)m * g.ldh + n] : 0.0f;
                }
    }
#pragma unroll
    for (int t = 0; t < G_NT; ++t) {
        if (kbeg + t * G_BK >= kend) break;  // uniform
        // two LDS buffers: the barrier after this store also orders every
        // wavefront's reads of buffer t & 1 two tiles ago before it
        bf16 (*As)[G_LD] = Ab[t & 1];
        bf16 (*Bs)[G_LD] = Bb[t & 1];
        regs[t].store(As, Bs, tid);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < G_BK; kk += 32) {
            const int kq = kk + 8 * (lane >> 4);
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
        }
    }
    float* C = g.C + (int64_t)bz * g.split_stride;
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
                    v += bias[j];
                    C[(int64_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_GELU) {
                    v += bias[j];
                    C[(int64_t)m * g.ldc + n] = v;
                    g.H[(int64_t)m * g.ldh + n] = f2bf(gelu_f(v));
                } else {
                    v *= gelu_grad_f(zin[i][j][r]);
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
            g.cs[(int64_t)by * g.N + n0 + tid] = cs_sh[0][tid] + cs_sh[1][tid];
    }
}

template <bool TA, bool TB, int EPI, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g)
{
    __shared__ __align__(16) bf16 As[2][G_BM][G_LD];
    __shared__ __align__(16) bf16 Bs[2][G_BN][G_LD];  // [n][k]
    __shared__ float cs_sh[2][G_BN];
    gemm_tile<TA, TB, EPI, VEC>(g, blockIdx.x, blockIdx.y, blockIdx.z, As, Bs, cs_sh);
}

// Two independent products in one launch (both VEC): workgroups [0, nb1) take
// the tiles of the first in (x, y, z) order, the rest those of the second.
template <bool TA1, bool TB1, int EPI1, bool TA2, bool TB2, int EPI2>
__global__ __launch_bounds__(256) void k_gemm_pair(GemmArgs g1, GemmArgs g2, int nb1)
{
    __shared__ __align__(16) bf16 As[2][G_BM][G_LD];
    __shared__ __align__(16) bf16 Bs[2][G_BN][G_LD];
    __shared__ float cs_sh[2][G_BN];
    int b = blockIdx.x;
    if (b < nb1) {
        gemm_tile<TA1, TB1, EPI1, true>(g1, b % g1.gx, (b / g1.gx) % g1.gy, b / (g1.gx * g1.gy), As, Bs, cs_sh);
    } else {
        b -= nb1;
        gemm_tile<TA2, TB2, EPI2, true>(g2, b % g2.gx, (b / g2.gx) % g2.gy, b / (g2.gx * g2.gy), As, Bs, cs_sh);
    }
}

// ----------------------------------------------------------------------------
// Output layer and loss in one pass: out = h2 W3 + b3 for 64 rows per
// workgroup, kept in LDS, then the mixture negative log-likelihood of each
// row and its gradient w.r.t. the 136 outputs (divided by the batch size, as
// bf16: the operand of both products that consume it).
// The loss (sum of NLL / batch) is accumulated atomically.
// ----------------------------------------------------------------------------
// Product: the workgroup's 64 rows of h2 and all of W3 (as its bf16
// transpose W3T [136][256], K contiguous) are loaded in one round trip and
// staged in LDS; wavefront w multiplies rows 16 w..16 w + 15 by the 9 column
// fragments (136 columns, padded to 144 with zeros) on
// v_mfma_f32_16x16x32_bf16 and writes them, plus b3, to its own LDS rows.
// Loss: 8 rows at a time per wavefront, lane 8 r + k holding row r's mixture
// component k (its logit, 8 means, 8 log sds, and the row's 8 targets), so
// the per-row sums over components are 8-lane shuffles and no lane repeats
// another's transcendentals. cs != null: the workgroup also writes the
// float32 column sums of its rows' gradient, cs[blockIdx][136] (the output
// bias's gradient partials).
constexpr int OL_ROWS = 64, OL_WAVES = 4, OL_LD = NN_H + 8, OL_NP = 144, OL_OLD = NN_OUT + 4;
static_assert(NN_K == 8 && NN_D == 8 && NN_OUT == 136 && NN_H == 256, "output layer layout");

__device__ __forceinline__ float sum8(float v)  // over the 8 lanes of a row
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

__device__ __forceinline__ float max8(float v)
{
    v = fmaxf(v, __shfl_xor(v, 1, 64));
    v = fmaxf(v, __shfl_xor(v, 2, 64));
    v = fmaxf(v, __shfl_xor(v, 4, 64));
    return v;
}

__device__ __forceinline__ float sum_rows(float v)  // over the 8 rows (lane bits 3..5)
{
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Orders one wavefront's LDS writes before its lanes read what other lanes
// wrote: a wavefront-scope fence pair around a wave barrier.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * OL_WAVES) void k_out_loss(const bf16* H2, const bf16* W3T, const float* b3,
                                                          const float* T, int n, bf16* dout_b,
                                                          float* loss_acc, const int32_t* step,
                                                          float* loss_log, float* cs)
{
    __shared__ __align__(16) bf16 As[OL_ROWS][OL_LD];
    __shared__ __align__(16) bf16 Bs[OL_NP][OL_LD];    // [n][k]
    __shared__ __align__(16) float Os[OL_ROWS][OL_OLD];
    __shared__ float red[OL_WAVES];
    __shared__ float csh[OL_WAVES][NN_OUT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.x * OL_ROWS;
    constexpr int KV = NN_H / 8;                              // 8-element vectors per row
    constexpr int NA = OL_ROWS * KV / 256, NB = NN_OUT * KV / 256;  // 8 and 17 per thread
    static_assert(OL_ROWS * KV % 256 == 0 && NN_OUT * KV % 256 == 0, "whole vectors per thread");
    const us8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    us8 va[NA], vb[NB];
#pragma unroll
    for (int h = 0; h < NA; ++h) {
        const int v = tid + 256 * h, r = v / KV, kv = v % KV;
        va[h] = m0 + r < n ? *reinterpret_cast<const us8*>(H2 + (int64_t)(m0 + r) * NN_H + kv * 8) : zero;
    }
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const int v = tid + 256 * h;
        vb[h] = *reinterpret_cast<const us8*>(W3T + (int64_t)(v / KV) * NN_H + (v % KV) * 8);
    }
    // the epilogue's biases and the loss's targets are requested with the operands
    float bias[OL_NP / 16];
#pragma unroll
    for (int f = 0; f < OL_NP / 16; ++f) {
        const int c = 16 * f + (lane & 15);
        bias[f] = c < NN_OUT ? b3[c] : 0.0f;
    }
    const int k = lane & 7;
    float4 tv[2][2];
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        const int row = m0 + 16 * wv + 8 * grp + (lane >> 3);
        const float4* t4 = reinterpret_cast<const float4*>(T + (int64_t)(row < n ? row : 0) * NN_D);
        tv[grp][0] = t4[0];
        tv[grp][1] = t4[1];
    }
#pragma unroll
    for (int h = 0; h < NA; ++h) {
        const int v = tid + 256 * h;
        *reinterpret_cast<us8*>(&As[v / KV][(v % KV) * 8]) = va[h];
    }
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const int v = tid + 256 * h;
        *reinterpret_cast<us8*>(&Bs[v / KV][(v % KV) * 8]) = vb[h];
    }
    static_assert((OL_NP - NN_OUT) * KV == 256, "one padding vector per thread");
    *reinterpret_cast<us8*>(&Bs[NN_OUT + tid / KV][(tid % KV) * 8]) = zero;
    __syncthreads();
    float4_t acc[OL_NP / 16];
#pragma unroll
    for (int f = 0; f < OL_NP / 16; ++f) acc[f] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < NN_H; kk += 32) {
        const int kq = kk + 8 * (lane >> 4);
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&As[16 * wv + (lane & 15)][kq]);
#pragma unroll
        for (int f = 0; f < OL_NP / 16; ++f) {
            const bf16x8 bf = *reinterpret_cast<const bf16x8*>(&Bs[16 * f + (lane & 15)][kq]);
            acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[f], 0, 0, 0);
        }
    }
#pragma unroll
    for (int f = 0; f < OL_NP / 16; ++f) {
        const int c = 16 * f + (lane & 15);
        if (c < NN_OUT) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Os[16 * wv + 4 * (lane >> 4) + r][c] = acc[f][r] + bias[f];
        }
    }
    wave_lds_sync();  // from here on the wavefront reads only its own rows

    const float inv_n = 1.0f / (float)n;
    float nll = 0.0f, ck = 0.0f, cm[8], cl[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) cm[j] = cl[j] = 0.0f;
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        const int rl = 16 * wv + 8 * grp + (lane >> 3);
        const int row = m0 + rl;
        const bool live = row < n;
        const float* o = &Os[rl][0];
        const float4* mu4 = reinterpret_cast<const float4*>(o + NN_K + NN_D * k);
        const float4* raw4 = reinterpret_cast<const float4*>(o + NN_K + NN_K * NN_D + NN_D * k);
        const float logit = o[k];
        const float4 m0v = mu4[0], m1v = mu4[1], r0v = raw4[0], r1v = raw4[1], t0v = tv[grp][0], t1v = tv[grp][1];
        const float mu[8] = {m0v.x, m0v.y, m0v.z, m0v.w, m1v.x, m1v.y, m1v.z, m1v.w};
        const float raw[8] = {r0v.x, r0v.y, r0v.z, r0v.w, r1v.x, r1v.y, r1v.z, r1v.w};
        const float t[8] = {t0v.x, t0v.y, t0v.z, t0v.w, t1v.x, t1v.y, t1v.z, t1v.w};
        // log-softmax of the row's logits
        const float lmax = max8(logit);
        const float lse_logits = lmax + logf(sum8(expf(logit - lmax)));
        // component k's log density: sum over dimensions of -u^2 / 2 - log sd
        float u[8], si[8], term = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float ls = fminf(fmaxf(raw[j], LOGSIG_LO), LOGSIG_HI);
            si[j] = expf(-ls);
            u[j] = (t[j] - mu[j]) * si[j];
            term += -0.5f * u[j] * u[j] - ls;
        }
        const float Lk = logit - lse_logits - 0.5f * NN_D * 1.83787706640934548356f + term;
        // log-sum-exp over the components
        const float Lmax = max8(Lk);
        const float lse = Lmax + logf(sum8(expf(Lk - Lmax)));
        const float resp = expf(Lk - lse);
        const float gk = live ? (expf(logit - lse_logits) - resp) * inv_n : 0.0f;
        float gmu[8], gls[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            gmu[j] = live ? -resp * u[j] * si[j] * inv_n : 0.0f;
            gls[j] = (live && raw[j] > LOGSIG_LO && raw[j] < LOGSIG_HI) ? -resp * (u[j] * u[j] - 1.0f) * inv_n
                                                                         : 0.0f;
        }
        if (live) {
            bf16* gb = dout_b + (int64_t)row * NN_OUT;
            gb[k] = f2bf(gk);
            us8 bm, bl;
#pragma unroll
            for (int j = 0; j < 8; ++j) { bm[j] = f2bf(gmu[j]); bl[j] = f2bf(gls[j]); }
            *reinterpret_cast<us8*>(gb + NN_K + NN_D * k) = bm;
            *reinterpret_cast<us8*>(gb + NN_K + NN_K * NN_D + NN_D * k) = bl;
        }
        if (live && k == 0) nll += -lse;
        ck += gk;
#pragma unroll
        for (int j = 0; j < 8; ++j) { cm[j] += gmu[j]; cl[j] += gls[j]; }
    }
    // the wavefront's loss (rows in lane order) and column sums (8 rows, fixed tree)
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) nll += __shfl_xor(nll, off, 64);
    if (lane == 0) red[wv] = nll;
    if (cs) {
        ck = sum_rows(ck);
#pragma unroll
        for (int j = 0; j < 8; ++j) { cm[j] = sum_rows(cm[j]); cl[j] = sum_rows(cl[j]); }
        if (lane < 8) {
            csh[wv][k] = ck;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                csh[wv][NN_K + NN_D * k + j] = cm[j];
                csh[wv][NN_K + NN_K * NN_D + NN_D * k + j] = cl[j];
            }
        }
    }
    __syncthreads();
    // one atomic per workgroup for the loss (its value only): into the log
    // entry of the counter's step when training, else into loss_acc
    float* dst = loss_log ? loss_log + *step : loss_acc;
    if (tid == 0 && dst) {
        float s = 0.0f;
        for (int w = 0; w < OL_WAVES; ++w) s += red[w];
        atomicAdd(dst, s / (float)n);
    }
    if (cs && tid < NN_OUT) {
        float s = 0.0f;
        for (int w = 0; w < OL_WAVES; ++w) s += csh[w][tid];
        cs[(int64_t)blockIdx.x * NN_OUT + tid] = s;
    }
}

// ----------------------------------------------------------------------------
// Adam (Kingma & Ba) on the float32 master parameters, then the bf16 copies
// of the weights
// ----------------------------------------------------------------------------
// The gradient of every parameter from its partials, added in fixed order:
// a weight entry from the split-K partials of its layer's product (split
// order), a bias entry from the column-sum partials of its layer (row-block
// order). With adam, the same thread then applies Adam to the float32 master
// parameter, at the update count the step counter holds (the first backward
// launch has advanced it), and refreshes its bf16 copy. With gather_rows > 0
// the workgroups after the parameters' assemble the next step's batch (two
// rows each) while the partials are summed: the step's products are done
// with X and T.
constexpr int FIN_PARAM_BLOCKS = (int)((NN_PARAMS + 255) / 256);

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
    int gather_rows;      // batch rows to assemble for the next step (0: none)
    int64_t steps_total;  // no batch is assembled once the counter reaches it
    RowMap rm;
    bf16* X;
    float* T;
};

__global__ __launch_bounds__(256) void k_grad_finish(FinishArgs a)
{
    if (blockIdx.x >= FIN_PARAM_BLOCKS) {
        const int st = *a.step;
        const int b = 2 * (blockIdx.x - FIN_PARAM_BLOCKS) + (threadIdx.x >> 7);
        if (st < a.steps_total && b < a.gather_rows) gather_row(a.rm, st, b, threadIdx.x & 127, a.X, a.T);
        return;
    }
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
    // Adam's state is requested before the partials are summed
    float m0 = 0.0f, v0 = 0.0f, p0 = 0.0f;
    if (a.adam) { m0 = a.m[e]; v0 = a.v[e]; p0 = a.p[e]; }
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
    const int st = *a.step;  // updates so far, this one included
    const float m = a.b1 * m0 + (1.0f - a.b1) * gsum;
    const float v = a.b2 * v0 + (1.0f - a.b2) * gsum * gsum;
    a.m[e] = m;
    a.v[e] = v;
    const float mh = m / (1.0f - powf(a.b1, (float)st));
    const float vh = v / (1.0f - powf(a.b2, (float)st));
    const float p = p0 - a.lr * mh / (sqrtf(vh) + a.eps);
    a.p[e] = p;
    put_bf16(a.pb, e, p);
}

__global__ void k_zero_f32(float* p, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.0f;
}

__global__ void k_params_bf16(const float* p, bf16* pb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < NN_PARAMS) put_bf16(pb, e, p[e]);
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
// batch): 128 rows per split once K >= 512, else K in ranges of at most
// G_KMAX.
static int k_per_split_for(int K)
{
    if (K >= 512) return 128;
    const int tiles = (K + G_BK - 1) / G_BK;
    const int splits = (tiles + G_NT - 1) / G_NT;
    return ((tiles + splits - 1) / splits) * G_BK;
}
static int splits_for(int K) { const int kps = k_per_split_for(K); return (K + kps - 1) / kps; }

// kps = K range per split (0: the whole K in one split); returns whether the
// operands allow the vector loads
template <bool TA, bool TB>
static bool gemm_prep(GemmArgs& g, int kps)
{
    g.k_per_split = kps > 0 ? kps : ((g.K + G_BK - 1) / G_BK) * G_BK;
    g.split_stride = (int64_t)g.M * g.N;
    g.gx = (g.N + G_BN - 1) / G_BN;
    g.gy = (g.M + G_BM - 1) / G_BM;
    return g.M % 8 == 0 && g.N % 8 == 0 && g.K % 8 == 0 && g.lda % 8 == 0 && g.ldb % 8 == 0 &&
           g.k_per_split % 8 == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15u) == 0 &&
           (reinterpret_cast<uintptr_t>(g.B) & 15u) == 0;
}

static int splits_of(const GemmArgs& g) { return (g.K + g.k_per_split - 1) / g.k_per_split; }

template <bool TA, bool TB, int EPI>
static void gemm(const GemmArgs& g0, int kps, hipStream_t s)
{
    GemmArgs g = g0;
    const bool vec = gemm_prep<TA, TB>(g, kps);
    const dim3 grid(g.gx, g.gy, splits_of(g));
    if (vec)
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, true>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, false>), grid, dim3(256), 0, s, g);
}

// two independent products in one launch where both allow vector loads
// (the first one's tiles are dispatched first), else one launch each
template <bool TA1, bool TB1, int EPI1, bool TA2, bool TB2, int EPI2>
static void gemm_pair(const GemmArgs& a0, int kps1, const GemmArgs& b0, int kps2, hipStream_t s)
{
    GemmArgs a = a0, b = b0;
    const bool va = gemm_prep<TA1, TB1>(a, kps1), vb = gemm_prep<TA2, TB2>(b, kps2);
    if (!va || !vb) {
        gemm<TA1, TB1, EPI1>(a0, kps1, s);
        gemm<TA2, TB2, EPI2>(b0, kps2, s);
        return;
    }
    const int na = a.gx * a.gy * splits_of(a), nb = b.gx * b.gy * splits_of(b);
    hipLaunchKernelGGL((k_gemm_pair<TA1, TB1, EPI1, TA2, TB2, EPI2>), dim3(na + nb), dim3(256), 0, s, a, b,
                       na);
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
    float *T = nullptr, *Z1 = nullptr, *Z2 = nullptr, *OUT = nullptr;
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
                    n->OUT, n->part1, n->part2, n->part3,
                    n->cs1, n->cs2, n->cs3};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    n->X = n->H1 = n->H2 = n->dOUTb = n->dZ2b = n->dZ1b = nullptr;
    n->T = n->Z1 = n->Z2 = n->OUT = nullptr;
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
    ALLOC(n->dOUTb, r * NN_OUT * sizeof(bf16));
    ALLOC(n->dZ2b, r * NN_H * sizeof(bf16));
    ALLOC(n->dZ1b, r * NN_H * sizeof(bf16));
    ALLOC(n->part1, (size_t)splits * NN_IN * NN_H * sizeof(float));
    ALLOC(n->part2, (size_t)splits * NN_H * NN_H * sizeof(float));
    ALLOC(n->part3, (size_t)splits * NN_H * NN_OUT * sizeof(float));
    ALLOC(n->cs1, (size_t)((rows + G_BM - 1) / G_BM) * NN_H * sizeof(float));
    ALLOC(n->cs2, (size_t)((rows + G_BM - 1) / G_BM) * NN_H * sizeof(float));
    ALLOC(n->cs3, (size_t)((rows + OL_ROWS - 1) / OL_ROWS) * NN_OUT * sizeof(float));
#undef ALLOC
    n->ws = rows;
    return ABC_OK;
}

// the batch's rows: rows 0..batch-1 in order without a step counter
RowMap row_map(const abc_mdn* net, const float* features, const float* theta, int64_t n_rows,
               int batch, int steps_per_epoch, const int64_t* perm, const int32_t* step)
{
    RowMap r{};
    r.features = features;
    r.theta = theta;
    r.n = n_rows;
    r.batch = batch;
    r.steps_per_epoch = steps_per_epoch;
    r.perm_ab = perm;
    r.step = step;
    r.fmean = net->fmean;
    r.fsd = net->fsd;
    for (int j = 0; j < 8; ++j) { r.tc[j] = net->tc[j]; r.ts[j] = net->ts[j]; }
    return r;
}

void launch_gather(abc_mdn* net, const RowMap& rm, int rows, float* loss_acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(rows), dim3(128), 0, s, rm, net->X, net->T, loss_acc);
}

// the hidden layers: Z1, H1, Z2, H2 from X
void forward_hidden(abc_mdn* net, int n, hipStream_t s)
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
}

// the network outputs OUT (inference)
void forward_out(abc_mdn* net, int n, hipStream_t s)
{
    GemmArgs g{};
    g.M = n; g.N = NN_OUT; g.K = NN_H;
    g.A = net->H2; g.lda = NN_H; g.B = net->pb + OFF_W3; g.ldb = NN_OUT;
    g.C = net->OUT; g.ldc = NN_OUT; g.bias = net->p + OFF_B3;
    gemm<false, false, EPI_STORE>(g, 0, s);
}

// output layer, loss and the gradient partials of the mean NLL
// (forward_hidden must have run); the gradient itself is formed by
// k_grad_finish. The weight gradient of a layer
// and the next layer's input gradient do not depend on each other and share
// a launch. Training (step != null): the loss goes to loss_log[step] and the
// first backward launch advances the step counter (no kernel of this launch
// reads it).
void backward(abc_mdn* net, int n, int32_t* step, float* loss_log, hipStream_t s)
{
    hipLaunchKernelGGL(k_out_loss, dim3((n + OL_ROWS - 1) / OL_ROWS), dim3(64 * OL_WAVES), 0, s, net->H2,
                       net->pb + OFF_W3T, net->p + OFF_B3, net->T, n, net->dOUTb, net->loss_acc, step,
                       step ? loss_log : nullptr, net->cs3);
    const int kps = k_per_split_for(n);
    // dZ2 = (dOUT W3^T) gelu'(Z2), with the column partials of db2; dW3 = H2^T dOUT
    // (db3: the loss kernel's column partials)
    GemmArgs d{}, w{};
    d.M = n; d.N = NN_H; d.K = NN_OUT;
    d.A = net->dOUTb; d.lda = NN_OUT; d.B = net->pb + OFF_W3; d.ldb = NN_OUT;
    d.Zin = net->Z2; d.H = net->dZ2b; d.ldh = NN_H; d.cs = net->cs2;
    d.step_inc = step;
    w.M = NN_H; w.N = NN_OUT; w.K = n;
    w.A = net->H2; w.lda = NN_H; w.B = net->dOUTb; w.ldb = NN_OUT;
    w.C = net->part3; w.ldc = NN_OUT;
    gemm_pair<false, true, EPI_DGELU, true, false, EPI_STORE>(d, 0, w, kps, s);
    // dZ1 = (dZ2 W2^T) gelu'(Z1), with the column partials of db1; dW2 = H1^T dZ2
    d = GemmArgs{};
    w = GemmArgs{};
    d.M = n; d.N = NN_H; d.K = NN_H;
    d.A = net->dZ2b; d.lda = NN_H; d.B = net->pb + OFF_W2; d.ldb = NN_H;
    d.Zin = net->Z1; d.H = net->dZ1b; d.ldh = NN_H; d.cs = net->cs1;
    w.M = NN_H; w.N = NN_H; w.K = n;
    w.A = net->H1; w.lda = NN_H; w.B = net->dZ2b; w.ldb = NN_H;
    w.C = net->part2; w.ldc = NN_H;
    gemm_pair<false, true, EPI_DGELU, true, false, EPI_STORE>(d, 0, w, kps, s);
    // dW1 = X^T dZ1
    w = GemmArgs{};
    w.M = NN_IN; w.N = NN_H; w.K = n;
    w.A = net->X; w.lda = NN_IN; w.B = net->dZ1b; w.ldb = NN_H;
    w.C = net->part1; w.ldc = NN_H;
    gemm<true, false, EPI_STORE>(w, kps, s);
}

FinishArgs finish_args(abc_mdn* net, int n)
{
    FinishArgs f{};
    f.part1 = net->part1; f.part2 = net->part2; f.part3 = net->part3;
    f.splits = splits_for(n);
    f.cs1 = net->cs1; f.cs2 = net->cs2; f.cs3 = net->cs3;
    f.tiles = (n + G_BM - 1) / G_BM;
    f.lblocks = (n + OL_ROWS - 1) / OL_ROWS;
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
    e = e ? e : hipMalloc((void**)&n->pb, NN_PB * sizeof(bf16));
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
    hipLaunchKernelGGL(k_params_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, 0, n->p, n->pb);
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
    hipLaunchKernelGGL(k_params_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, as_stream(stream), n->p, n->pb);
    return check_launch("k_params_bf16");
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
    ABC_REQUIRE((reinterpret_cast<uintptr_t>(features) & 15u) == 0, "features must be 16-byte aligned");
    abc_status rc = ensure_ws(net, (int)n);
    if (rc) return rc;
    const hipStream_t s = as_stream(stream);
    launch_gather(net, row_map(net, features, nullptr, n, (int)n, 1, nullptr, nullptr), (int)n, nullptr, s);
    forward_hidden(net, (int)n, s);
    forward_out(net, (int)n, s);
    ABC_HIP(hipMemcpyAsync(out, net->OUT, (size_t)n * NN_OUT * sizeof(float), hipMemcpyDeviceToDevice, s));
    return check_launch("abc_mdn_forward");
}

extern "C" abc_status abc_mdn_loss_grad(abc_mdn* net, const float* features, const float* theta,
                                        int64_t n, float* loss, float* grad, void* stream)
{
    ABC_REQUIRE(net && features && theta && n >= 1 && n <= (1 << 20), "bad arguments");
    ABC_REQUIRE((reinterpret_cast<uintptr_t>(features) & 15u) == 0, "features must be 16-byte aligned");
    abc_status rc = ensure_ws(net, (int)n);
    if (rc) return rc;
    const hipStream_t s = as_stream(stream);
    launch_gather(net, row_map(net, features, theta, n, (int)n, 1, nullptr, nullptr), (int)n, net->loss_acc, s);
    forward_hidden(net, (int)n, s);
    backward(net, (int)n, nullptr, nullptr, s);
    const FinishArgs f = finish_args(net, (int)n);
    hipLaunchKernelGGL(k_grad_finish, dim3(FIN_PARAM_BLOCKS), dim3(256), 0, s, f);
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
    ABC_REQUIRE((reinterpret_cast<uintptr_t>(features) & 15u) == 0, "features must be 16-byte aligned");
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
    if (loss_log) ABC_HIP(hipMemsetAsync(loss_log, 0, (size_t)steps * sizeof(float), s));
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->m, NN_PARAMS);
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->v, NN_PARAMS);
    // the first batch; every step's finish kernel assembles the next one
    const RowMap rm = row_map(net, features, theta, n, batch, spe, net->perm, net->step);
    launch_gather(net, rm, batch, nullptr, s);
    ABC_HIP(hipStreamSynchronize(s));

    // one training step, captured once and replayed
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ABC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    forward_hidden(net, batch, s);
    backward(net, batch, net->step, loss_log, s);
    FinishArgs f = finish_args(net, batch);
    f.adam = 1;
    f.p = net->p; f.m = net->m; f.v = net->v; f.pb = net->pb; f.step = net->step;
    f.lr = lr; f.b1 = 0.9f; f.b2 = 0.999f; f.eps = 1e-8f;
    f.gather_rows = batch;
    f.steps_total = steps;
    f.rm = rm;
    f.X = net->X;
    f.T = net->T;
    hipLaunchKernelGGL(k_grad_finish, dim3(FIN_PARAM_BLOCKS + (batch + 1) / 2), dim3(256), 0, s, f);
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
    hipLaunchKernelGGL(k_params_bf16, dim3(blocks_for(NN_PARAMS)), dim3(256), 0, s, net->p, net->pb);
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
