// ABC-SMC: population Monte Carlo ABC over a decreasing tolerance sequence
// (Sec. 2.2 names the method; the algorithm is that of Beaumont, Cornuet,
// Marin & Robert, Biometrika 2009, with the adaptive quantile tolerance of
// Del Moral, Doucet & Jasra, Stat. Comput. 2012), and its C-ABI entry points
// abc_smc_generation and abc_smc_run.
//
// One generation t >= 1 on the device:
//   k_smc_setup     one workgroup: weighted mean and covariance of generation
//                   t-1 (left-to-right float64 sums), Sigma = 2 cov, its
//                   Cholesky factor L, running weight sums C_j, whitened
//                   particles y_j = L^-1 theta_j, and eps_t, the kth smallest
//                   previous distance, by radix selection.
//   k_smc_propose   one lane per candidate: ancestor by binary search of
//                   u C_{N-1} in C, theta* = theta_anc + L z (float64, rounded
//                   to float32).
//   simulate / compact / float64 decision: the rejection-ABC kernels, with
//                   the prior-support check (candidates outside the box are
//                   rejected unsimulated); with a band every candidate is
//                   decided by its float64 distance; the first N accepted by
//                   index form the population.
//   float64 distances of the population (for eps_{t+1}): with a band, the
//                   float64 decision runs on every candidate (alone on the GPU,
//                   rows side by side cost no more latency than the band's) and
//                   its distances are kept; without one, abc_simulate_rows_f64.
//   k_smc_sums      importance-weight denominators sum_j W_j exp(-|y_i - y_j|^2 / 2),
//                   split over the previous particles for parallelism.
//   k_smc_finish    w_i = 1 / denominator, W = w / sum w (left to right), ESS.
// Generation 0 is plain rejection ABC from the prior on the ABC stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "model.hpp"
#include "philox.hpp"

namespace abc {

constexpr int SMC_MAX_N = 8192;
constexpr uint32_t DOMAIN_SMC = 7;
constexpr uint32_t DOMAIN_ABC_PLAIN = 1;

struct SmcState {
    double L[64];     // row-major, lower triangle
    double mean[8];
    double sigma[64]; // 2 x weighted covariance
    double total;     // C_{N-1}
    double eps64;     // order statistic before the floor and the float32 rounding
    float eps;
    int32_t status;   // 0 ok, 1 Sigma not positive definite
};

struct SetupArgs {
    const float* theta;   // [N][8]
    const double* w;      // [N] normalised weights
    const double* dist;   // [N] float64 distances
    int32_t N;
    int32_t kth;          // ceil(alpha N), 1-based
    float eps_min;
    SmcState* st;
    double* C;            // [N]
    double* y;            // [N][8]
};

// The single-lane ordered sums read the particles from LDS: all threads copy
// a chunk of SMC_CHUNK particles (weights, then theta) into the distance
// array before it holds the distances, and the summing lanes load SMC_PF
// values ahead of their adds. The order of the additions is that of the
// plainly written definition.
constexpr int SMC_PF = 16;
constexpr int SMC_CHUNK = 1024;  // 8 KiB of weights + 32 KiB of theta

__device__ __forceinline__ void smc_stage_chunk(const SetupArgs& a, int c0, int m, double* sw,
                                                float* sth)
{
    // one particle per thread: all nine loads are in flight before any store
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const float* src = a.theta + (int64_t)8 * (c0 + j);
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = src[k];
        const double wj = a.w[c0 + j];
        sw[j] = wj;
#pragma unroll
        for (int k = 0; k < 8; ++k) sth[8 * j + k] = v[k];
    }
}

// Keys whose unsigned order is the order of the (non-NaN) doubles.
__device__ __forceinline__ uint64_t order_key(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ __forceinline__ double key_value(uint64_t k)
{
    const uint64_t b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
    return __longlong_as_double((long long)b);
}

constexpr int SMC_SETUP_THREADS = 1024;
constexpr int SMC_SEL_PER = SMC_MAX_N / SMC_SETUP_THREADS;

// One workgroup of SMC_SETUP_THREADS threads. Sums run left to right over the
// particles in single lanes so that every rounding matches the plainly written
// definition.
__global__ __launch_bounds__(SMC_SETUP_THREADS) void k_smc_setup(SetupArgs a)
{
#pragma clang fp contract(off)
    __shared__ double sd[SMC_MAX_N];
    __shared__ double m_sh[8];
    __shared__ double v_sh;
    __shared__ double sig_sh[64];
    __shared__ unsigned long long sel_prefix;
    __shared__ unsigned int sel_rank;
    __shared__ double l_sh[64];
    __shared__ int status_sh;
    static_assert(SMC_CHUNK * 6 <= SMC_MAX_N, "staging chunk exceeds the distance array");
    double* sw = sd;
    float* sth = reinterpret_cast<float*>(sd + SMC_CHUNK);
    double* sC = sd + 5 * SMC_CHUNK;  // running sums of the chunk, stored coalesced
    const int tid = threadIdx.x;
    const int N = a.N;
    // phase A: running weight sums (lane 64), sums of W theta (lanes 0..7)
    double sc = 0.0, sm = 0.0;
    for (int c0 = 0; c0 < N; c0 += SMC_CHUNK) {
        const int m = min(SMC_CHUNK, N - c0);
        smc_stage_chunk(a, c0, m, sw, sth);
        __syncthreads();
        if (tid == 64) {
            int j = 0;
            for (; j + SMC_PF <= m; j += SMC_PF) {
                double wv[SMC_PF];
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) wv[k] = sw[j + k];
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) {
                    sc = sc + wv[k];
                    sC[j + k] = sc;
                }
            }
            for (; j < m; ++j) {
                sc = sc + sw[j];
                sC[j] = sc;
            }
        }
        if (tid < 8) {
            int j = 0;
            for (; j + SMC_PF <= m; j += SMC_PF) {
                double wv[SMC_PF];
                float tv[SMC_PF];
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) {
                    wv[k] = sw[j + k];
                    tv[k] = sth[8 * (j + k) + tid];
                }
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) sm = sm + wv[k] * (double)tv[k];
            }
            for (; j < m; ++j) sm = sm + sw[j] * (double)sth[8 * j + tid];
        }
        __syncthreads();
        for (int j = tid; j < m; j += blockDim.x) a.C[c0 + j] = sC[j];
    }
    if (tid == 64) {
        v_sh = sc;
        a.st->total = sc;
    }
    __syncthreads();
    if (tid < 8) {
        m_sh[tid] = sm / v_sh;
        a.st->mean[tid] = m_sh[tid];
    }
    __syncthreads();
    // phase B: covariance entries (a >= b), one lane each
    int r = 0, c = 0;
    double mr = 0.0, mc = 0.0, sv = 0.0;
    if (tid < 36) {
        while ((r + 1) * (r + 2) / 2 <= tid) ++r;
        c = tid - r * (r + 1) / 2;
        mr = m_sh[r];
        mc = m_sh[c];
    }
    for (int c0 = 0; c0 < N; c0 += SMC_CHUNK) {
        const int m = min(SMC_CHUNK, N - c0);
        smc_stage_chunk(a, c0, m, sw, sth);
        __syncthreads();
        if (tid < 36) {
            int j = 0;
            for (; j + SMC_PF <= m; j += SMC_PF) {
                double wv[SMC_PF];
                float tr[SMC_PF], tc[SMC_PF];
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) {
                    wv[k] = sw[j + k];
                    tr[k] = sth[8 * (j + k) + r];
                    tc[k] = sth[8 * (j + k) + c];
                }
#pragma unroll
                for (int k = 0; k < SMC_PF; ++k) {
                    const double dr = (double)tr[k] - mr;
                    const double dc = (double)tc[k] - mc;
                    sv = sv + wv[k] * (dr * dc);
                }
            }
            for (; j < m; ++j) {
                const double dr = (double)sth[8 * j + r] - mr;
                const double dc = (double)sth[8 * j + c] - mc;
                sv = sv + sw[j] * (dr * dc);
            }
        }
        __syncthreads();  // the chunk is replaced next
    }
    if (tid < 36) {
        const double sg = 2.0 * (sv / v_sh);
        a.st->sigma[8 * r + c] = sg;
        a.st->sigma[8 * c + r] = sg;
        sig_sh[8 * r + c] = sg;
    }
    // previous distances as order-preserving 64-bit keys, SMC_SEL_PER per thread
    uint64_t key[SMC_SEL_PER];
#pragma unroll
    for (int e = 0; e < SMC_SEL_PER; ++e) {
        const int j = tid + e * SMC_SETUP_THREADS;
        key[e] = j < N ? order_key(a.dist[j]) : 0ull;
    }
    __syncthreads();
    // phase C: Cholesky-Banachiewicz, row by row (lane 0). Fully unrolled so
    // that L stays in registers; nothing is assigned after the first
    // non-positive pivot, which sets the status.
    if (tid == 0) {
        double L[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) L[i] = 0.0;
        int bad = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double s = sig_sh[8 * i + j];
#pragma unroll
                for (int k = 0; k < j; ++k) s = s - L[8 * i + k] * L[8 * j + k];
                if (!bad) {
                    if (i == j) {
                        if (!(s > 0.0))
                            bad = 1;
                        else
                            L[8 * i + i] = sqrt(s);
                    } else {
                        L[8 * i + j] = s / L[8 * j + j];
                    }
                }
            }
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            a.st->L[i] = L[i];
            l_sh[i] = L[i];
        }
        a.st->status = bad;
        status_sh = bad;
    }
    // phase D: eps_t is the kth smallest previous distance: radix selection
    // over the keys, 8 bits per pass from the most significant, with one
    // histogram per wavefront in LDS (the distance array is free by now).
    {
        unsigned int* hist = reinterpret_cast<unsigned int*>(sd);  // [16][256]
        uint64_t prefix = 0;
        unsigned int rank = (unsigned int)a.kth;  // 1-based, among keys matching prefix
        for (int shift = 56; shift >= 0; shift -= 8) {
            for (int b = tid; b < 16 * 256; b += SMC_SETUP_THREADS) hist[b] = 0u;
            __syncthreads();
            const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
            unsigned int* hw = hist + 256 * (tid >> 6);
#pragma unroll
            for (int e = 0; e < SMC_SEL_PER; ++e) {
                const int j = tid + e * SMC_SETUP_THREADS;
                if (j < N && (key[e] & hmask) == prefix)
                    atomicAdd(&hw[(unsigned)(key[e] >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid < 64) {
                unsigned int c[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    unsigned int t = 0;
                    for (int w = 0; w < 16; ++w) t += hist[256 * w + 4 * tid + q];
                    c[q] = t;
                }
                const unsigned int tot = c[0] + c[1] + c[2] + c[3];
                unsigned int incl = tot;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const unsigned int v = __shfl_up(incl, o, 64);
                    if (tid >= o) incl += v;
                }
                const unsigned int excl = incl - tot;
                if (excl < rank && rank <= incl) {
                    unsigned int run = excl;
                    int q = 0;
                    while (q < 3 && run + c[q] < rank) run += c[q++];
                    sel_prefix = prefix | ((uint64_t)(4 * tid + q) << shift);
                    sel_rank = rank - run;
                }
            }
            __syncthreads();
            prefix = sel_prefix;
            rank = sel_rank;
        }
        if (tid == 0) {
            const double q = key_value(prefix);
            a.st->eps64 = q;
            const double f = (double)a.eps_min;
            a.st->eps = (float)(q > f ? q : f);
        }
    }
    __syncthreads();
    // phase E: whitened particles y_j = L^-1 theta_j (forward substitution)
    if (status_sh == 0) {
        double L[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) L[i] = l_sh[i];
        for (int j = tid; j < N; j += blockDim.x) {
            double yv[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                double s = (double)a.theta[8 * j + r];
#pragma unroll
                for (int k = 0; k < r; ++k) s = s - L[8 * r + k] * yv[k];
                yv[r] = s / L[8 * r + r];
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) a.y[8 * j + r] = yv[r];
        }
    }
}

struct ProposeArgs {
    Key key;
    uint32_t series;      // series | gen << 16
    uint64_t first;
    int64_t n;
    const float* prev;    // [N][8]
    const double* C;      // [N]
    int32_t N;
    const SmcState* st;
    float* theta;         // [n][8]
    int32_t* anc;         // [n] or null
};

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1)
{
#pragma clang fp contract(off)
    const double u1 = ((double)a + 1.0) * 0x1p-32;
    const double r = sqrt(-2.0 * log(u1));
    const double phi = 6.283185307179586 * ((double)b * 0x1p-32);
    z0 = r * cos(phi);
    z1 = r * sin(phi);
}

__global__ __launch_bounds__(256) void k_smc_propose(ProposeArgs a)
{
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;
    const uint4 w0 = stream_words(a.key, i, a.series, ctr_word3(0, DOMAIN_SMC, 0));
    const uint4 w1 = stream_words(a.key, i, a.series, ctr_word3(0, DOMAIN_SMC, 1));
    const uint4 w2 = stream_words(a.key, i, a.series, ctr_word3(0, DOMAIN_SMC, 2));
    const double u = (double)(((uint64_t)w0.x << 21) | (uint64_t)(w0.y >> 11)) * 0x1p-53;
    double z[8];
    box_muller(w0.z, w0.w, z[0], z[1]);
    box_muller(w1.x, w1.y, z[2], z[3]);
    box_muller(w1.z, w1.w, z[4], z[5]);
    box_muller(w2.x, w2.y, z[6], z[7]);
    // smallest j with C_j > u C_{N-1}
    const double target = u * a.C[a.N - 1];
    int lo = 0, hi = a.N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.C[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    const int j = lo < a.N ? lo : a.N - 1;
    float out[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        double acc = (double)a.prev[8 * j + r];
#pragma unroll
        for (int c = 0; c <= r; ++c) acc = acc + a.st->L[8 * r + c] * z[c];
        out[r] = (float)acc;
    }
    float4* p = reinterpret_cast<float4*>(a.theta + 8 * k);
    p[0] = make_float4(out[0], out[1], out[2], out[3]);
    p[1] = make_float4(out[4], out[5], out[6], out[7]);
    if (a.anc) a.anc[k] = j;
}

__global__ void k_smc_zero_u64(unsigned long long* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// Number of rows of theta [m][8] inside the closed box (added to *count).
// Candidates inside the prior box: grid-stride count, one atomic per workgroup.
constexpr int BOX_GRID = 1024;

__global__ __launch_bounds__(256) void k_smc_count_box(const float* theta, int64_t m, abc_prior box,
                                                       unsigned long long* count)
{
    __shared__ unsigned int part[4];
    unsigned int c = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x) {
        const float4* p = reinterpret_cast<const float4*>(theta + 8 * k);
        const float4 u = p[0], v = p[1];
        const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
        bool in = true;
#pragma unroll
        for (int j = 0; j < 8; ++j) in &= x[j] >= box.lo[j] && x[j] <= box.hi[j];
        c += in ? 1u : 0u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        if (t) atomicAdd(count, t);
    }
}

// ancestors of the kept candidate rows (row r is candidate oidx[r] - first of the chunk)
__global__ __launch_bounds__(256) void k_smc_gather_anc(const int64_t* oidx, int64_t take, int64_t first,
                                                        const int32_t* anc_chunk, int32_t* out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < take) out[r] = anc_chunk[oidx[r] - first];
}

struct SumsArgs {
    const float* theta;   // new population [N][8]
    int32_t N;
    const double* y;      // previous, whitened [Np][8]
    const double* w;      // previous normalised weights [Np]
    int32_t Np;
    int32_t per_split;    // previous particles per blockIdx.y
    const SmcState* st;
    double* partial;      // [splits][N]
};

constexpr int SUMS_BLOCK = 256;

__global__ __launch_bounds__(SUMS_BLOCK) void k_smc_sums(SumsArgs a)
{
    __shared__ double ys[SUMS_BLOCK][9];  // y_j (8) and W_j
    const int i = blockIdx.x * SUMS_BLOCK + threadIdx.x;
    const int j0 = blockIdx.y * a.per_split;
    const int j1 = min(j0 + a.per_split, a.Np);
    double yi[8];
    if (i < a.N) {
        const double* L = a.st->L;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            double s = (double)a.theta[8 * i + r];
#pragma unroll
            for (int c = 0; c < r; ++c) s -= L[8 * r + c] * yi[c];
            yi[r] = s / L[8 * r + r];
        }
    }
    double acc = 0.0;
    for (int t0 = j0; t0 < j1; t0 += SUMS_BLOCK) {
        const int j = t0 + threadIdx.x;
        if (j < j1) {
#pragma unroll
            for (int r = 0; r < 8; ++r) ys[threadIdx.x][r] = a.y[8 * j + r];
            ys[threadIdx.x][8] = a.w[j];
        }
        __syncthreads();
        const int m = min(SUMS_BLOCK, j1 - t0);
        if (i < a.N)
            for (int jj = 0; jj < m; ++jj) {
                double q = 0.0;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const double d = yi[r] - ys[jj][r];
                    q = fma(d, d, q);
                }
                acc = fma(ys[jj][8], exp(-0.5 * q), acc);
            }
        __syncthreads();
    }
    if (i < a.N) a.partial[(int64_t)blockIdx.y * a.N + i] = acc;
}

// w_i = 1 / sum_s partial[s][i]; W = w / (w_0 + ... + w_{N-1}); ESS = 1 / sum W^2.
// The w_i stay in LDS for the single-lane left-to-right sum.
__global__ __launch_bounds__(1024) void k_smc_finish(const double* partial, int32_t splits,
                                                     int32_t N, double* W, double* ess)
{
#pragma clang fp contract(off)
    __shared__ double v_sh;
    __shared__ double wl[SMC_MAX_N];
    static_assert(SMC_MAX_N >= 1024, "the reduction reuses the weight array");
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s = 0.0;
        for (int sp = 0; sp < splits; ++sp) s = s + partial[(int64_t)sp * N + i];
        wl[i] = 1.0 / s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        int i = 0;
        for (; i + SMC_PF <= N; i += SMC_PF) {
            double v[SMC_PF];
#pragma unroll
            for (int k = 0; k < SMC_PF; ++k) v[k] = wl[i + k];
#pragma unroll
            for (int k = 0; k < SMC_PF; ++k) s = s + v[k];
        }
        for (; i < N; ++i) s = s + wl[i];
        v_sh = s;
    }
    __syncthreads();
    double q = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double x = wl[i] / v_sh;
        W[i] = x;
        q = q + x * x;
    }
    __syncthreads();  // every wl[i] has been read before the reduction reuses it
    double* red = wl;
    red[threadIdx.x] = q;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *ess = 1.0 / red[0];
}

__global__ __launch_bounds__(256) void k_smc_equal(double* W, int32_t N, double* ess)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) W[i] = 1.0 / (double)N;
    if (i == 0) *ess = (double)N;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static abc_status check_cfg(const abc_smc_config* c)
{
    ABC_REQUIRE(c != nullptr, "config is NULL");
    ABC_REQUIRE(c->n_particles >= 2 && c->n_particles <= SMC_MAX_N, "n_particles must be in [2, %d]",
                SMC_MAX_N);
    ABC_REQUIRE(c->generations >= 1 && c->generations <= 65535, "generations must be in [1, 65535]");
    ABC_REQUIRE(c->alpha > 0.0 && c->alpha <= 1.0, "alpha must be in (0, 1]");
    ABC_REQUIRE(isfinite(c->eps0) && c->eps0 >= 0.0f, "eps0 must be finite and >= 0");
    ABC_REQUIRE(isfinite(c->eps_min) && c->eps_min >= 0.0f, "eps_min must be finite and >= 0");
    ABC_REQUIRE(isfinite(c->band_w) && c->band_w >= 0.0f && c->band_w < 1.0f, "band_w must be in [0, 1)");
    ABC_REQUIRE(c->chunk0 >= 1 && c->chunk_max >= c->chunk0 && c->chunk_max <= ((int64_t)1 << 26),
                "need 1 <= chunk0 <= chunk_max <= 2^26");
    ABC_REQUIRE(c->max_samples >= 1, "max_samples must be >= 1");
    return ABC_OK;
}

static abc_status sync(hipStream_t s)
{
    ABC_HIP(hipStreamSynchronize(s));
    return ABC_OK;
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_smc_generation(const abc_series* ser, const abc_model* model,
                                         const abc_prior* prior, uint64_t seed, uint32_t series,
                                         int32_t gen, const float* prev_theta,
                                         const double* prev_w, const double* prev_dist,
                                         int32_t n_prev, const abc_smc_config* cfg, int64_t* idx,
                                         float* theta, double* w, double* dist,
                                         abc_smc_gen_stats* stats, int32_t* ancestors,
                                         void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    float lo[8], width[8];
    if ((rc = prior_lo_width(prior, lo, width))) return rc;
    for (int k = 0; k < 8; ++k)
        ABC_REQUIRE(prior->lo[k] >= 0.0f, "model rates must be non-negative: prior lo[%d] < 0", k);
    ABC_REQUIRE(series < 65536u, "series must be < 65536 (the generation shares its counter word)");
    ABC_REQUIRE(gen >= 0 && gen <= 65535, "gen must be in [0, 65535]");
    ABC_REQUIRE(idx && theta && w && dist && stats, "NULL output");
    ABC_REQUIRE((reinterpret_cast<uintptr_t>(theta) & 15u) == 0, "theta must be 16-byte aligned");
    if (gen > 0) {
        ABC_REQUIRE(prev_theta && prev_w && prev_dist, "generation >= 1 needs the previous population");
        ABC_REQUIRE(n_prev >= 2 && n_prev <= SMC_MAX_N, "n_prev must be in [2, %d]", SMC_MAX_N);
    }
    ABC_REQUIRE(!(model->flags & ABC_FP64), "ABC-SMC runs the float32 path with the float64 band decision");
    const hipStream_t s = as_stream(stream);
    const int N = cfg->n_particles;
    const int64_t cap = cfg->chunk_max;
    const uint32_t ss = gen == 0 ? series : (series | ((uint32_t)gen << 16));
    const abc_stream st{seed, gen == 0 ? DOMAIN_ABC_PLAIN : DOMAIN_SMC, ss};
    abc_model md = *model;
    if (gen > 0) md.flags |= ABC_SUPPORT;

    // workspace
    const int np = gen > 0 ? n_prev : 1;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_state = 0;
    const size_t o_C = o_state + up(sizeof(SmcState));
    const size_t o_y = o_C + up(sizeof(double) * np);
    const size_t o_cth = o_y + up(sizeof(double) * 8 * np);
    const size_t o_cd = o_cth + up(sizeof(float) * 8 * cap);
    const size_t o_oidx = o_cd + up(sizeof(float) * cap);
    const size_t o_oth = o_oidx + up(sizeof(int64_t) * cap);
    const size_t o_od = o_oth + up(sizeof(float) * 8 * cap);
    const size_t o_od64 = o_od + up(sizeof(float) * cap);
    const size_t o_cnt = o_od64 + up(sizeof(double) * cap);
    const size_t o_box = o_cnt + 256;
    const size_t o_ess = o_box + 256;
    const size_t o_anc = o_ess + 256;
    const size_t total = o_anc + up(sizeof(int32_t) * cap);
    void* ws = nullptr;
    if ((rc = stream_scratch(s, total, &ws, SCRATCH_SMC_WS))) return rc;
    char* base = static_cast<char*>(ws);
    SmcState* dstate = reinterpret_cast<SmcState*>(base + o_state);
    double* dC = reinterpret_cast<double*>(base + o_C);
    double* dy = reinterpret_cast<double*>(base + o_y);
    float* cth = reinterpret_cast<float*>(base + o_cth);
    float* cd = reinterpret_cast<float*>(base + o_cd);
    int64_t* oidx = reinterpret_cast<int64_t*>(base + o_oidx);
    float* oth = reinterpret_cast<float*>(base + o_oth);
    float* od = reinterpret_cast<float*>(base + o_od);
    double* od64 = reinterpret_cast<double*>(base + o_od64);
    int64_t* dcnt = reinterpret_cast<int64_t*>(base + o_cnt);
    unsigned long long* dbox = reinterpret_cast<unsigned long long*>(base + o_box);
    double* dess = reinterpret_cast<double*>(base + o_ess);
    int32_t* danc = reinterpret_cast<int32_t*>(base + o_anc);

    float eps = cfg->eps0;
    if (gen > 0) {
        SetupArgs sa{};
        sa.theta = prev_theta;
        sa.w = prev_w;
        sa.dist = prev_dist;
        sa.N = n_prev;
        int kth = (int)ceil(cfg->alpha * (double)n_prev);
        sa.kth = kth < 1 ? 1 : (kth > n_prev ? n_prev : kth);
        sa.eps_min = cfg->eps_min;
        sa.st = dstate;
        sa.C = dC;
        sa.y = dy;
        hipLaunchKernelGGL(k_smc_setup, dim3(1), dim3(SMC_SETUP_THREADS), 0, s, sa);
        if ((rc = check_launch("k_smc_setup"))) return rc;
        struct {
            float eps;
            int32_t status;
        } h{};
        ABC_HIP(hipMemcpyAsync(&h, &dstate->eps, sizeof h, hipMemcpyDeviceToHost, s));
        if ((rc = sync(s))) return rc;
        if (h.status)
            return set_error(ABC_EINVAL, "generation %d: kernel covariance of the previous population "
                             "is not positive definite", gen);
        eps = h.eps;
    }
    hipLaunchKernelGGL(k_smc_zero_u64, dim3(1), dim3(64), 0, s, dbox);

    const float e_hi = cfg->band_w > 0.0f ? (float)((double)eps * (1.0 + (double)cfg->band_w)) : eps;
    int got = 0;
    int64_t first = 0, chunk = cfg->chunk0, proposed = 0, samples = 0;
    while (got < N) {
        if (first >= cfg->max_samples)
            return set_error(ABC_EOVERFLOW, "generation %d: %d of %d particles after %lld candidates",
                             gen, got, N, (long long)first);
        const float* th_in = nullptr;
        if (gen > 0) {
            ProposeArgs pa{};
            pa.key = make_key(seed);
            pa.series = ss;
            pa.first = (uint64_t)first;
            pa.n = chunk;
            pa.prev = prev_theta;
            pa.C = dC;
            pa.N = n_prev;
            pa.st = dstate;
            pa.theta = cth;
            pa.anc = ancestors ? danc : nullptr;
            hipLaunchKernelGGL(k_smc_propose, dim3((unsigned)((chunk + 255) / 256)), dim3(256), 0, s, pa);
            if ((rc = check_launch("k_smc_propose"))) return rc;
            th_in = cth;
        }
        if ((rc = abc_simulate_distance(ser, &md, &st, th_in, prior, (uint64_t)first, chunk, e_hi, cd,
                                        nullptr, nullptr, stream)))
            return rc;
        if ((rc = abc_accept_compact(cd, th_in, nullptr, prior, &st, chunk, (uint64_t)first, e_hi, cap,
                                     oidx, oth, od, nullptr, dcnt, stream)))
            return rc;
        if (cfg->band_w > 0.0f &&
            (rc = recheck_band(ser, &md, &st, eps, cfg->band_w, cap, oidx, oth, od, nullptr, dcnt,
                               nullptr, stream, ROW_LDS_ALONE, ROW_WAVE_TARGET, ROW_SCAN_ALONE,
                               od64, true)))
            return rc;
        int64_t c = 0;
        ABC_HIP(hipMemcpyAsync(&c, dcnt, sizeof c, hipMemcpyDeviceToHost, s));
        if ((rc = sync(s))) return rc;
        if (c > cap) return set_error(ABC_EOVERFLOW, "candidate count %lld exceeds chunk_max", (long long)c);
        const int take = (int)(c < (int64_t)(N - got) ? c : (int64_t)(N - got));
        int64_t used = chunk;  // candidates of this chunk that the population consumes
        if (take > 0) {
            ABC_HIP(hipMemcpyAsync(idx + got, oidx, sizeof(int64_t) * take, hipMemcpyDeviceToDevice, s));
            ABC_HIP(hipMemcpyAsync(theta + 8 * (size_t)got, oth, sizeof(float) * 8 * take,
                                   hipMemcpyDeviceToDevice, s));
            if (cfg->band_w > 0.0f)
                ABC_HIP(hipMemcpyAsync(dist + got, od64, sizeof(double) * take,
                                       hipMemcpyDeviceToDevice, s));
            if (gen > 0 && ancestors) {
                hipLaunchKernelGGL(k_smc_gather_anc, dim3((unsigned)((take + 255) / 256)), dim3(256), 0,
                                   s, oidx, take, first, danc, ancestors + got);
                if ((rc = check_launch("k_smc_gather_anc"))) return rc;
            }
        }
        if (got + take == N) {
            int64_t last = 0;
            ABC_HIP(hipMemcpyAsync(&last, oidx + take - 1, sizeof last, hipMemcpyDeviceToHost, s));
            if ((rc = sync(s))) return rc;
            samples = last + 1;
            used = samples - first;
        }
        if (gen > 0) {
            const int64_t bb = (used + 255) / 256;
            hipLaunchKernelGGL(k_smc_count_box, dim3((unsigned)(bb < BOX_GRID ? bb : BOX_GRID)),
                               dim3(256), 0, s, cth, used, *prior, dbox);
            if ((rc = check_launch("k_smc_count_box"))) return rc;
        }
        got += take;
        proposed += chunk;
        first += chunk;
        chunk = chunk * 2 < cfg->chunk_max ? chunk * 2 : cfg->chunk_max;
    }

    // float64 distances of the population: with a band, the float64 decision
    // of every candidate has already produced them
    if (cfg->band_w <= 0.0f &&
        (rc = abc_simulate_rows_f64(ser, model, &st, idx, theta, N, dist, stream)))
        return rc;
    // weights
    if (gen == 0) {
        hipLaunchKernelGGL(k_smc_equal, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w, N, dess);
        if ((rc = check_launch("k_smc_equal"))) return rc;
    } else {
        const int bx = (N + SUMS_BLOCK - 1) / SUMS_BLOCK;
        int splits = 2048 / bx;
        const int max_splits = (n_prev + SUMS_BLOCK - 1) / SUMS_BLOCK;
        if (splits > max_splits) splits = max_splits;
        if (splits < 1) splits = 1;
        const int per = (n_prev + splits - 1) / splits;
        void* part = nullptr;
        if ((rc = stream_scratch(s, sizeof(double) * (size_t)splits * N, &part, SCRATCH_SMC_SUMS)))
            return rc;
        SumsArgs sa{};
        sa.theta = theta;
        sa.N = N;
        sa.y = dy;
        sa.w = prev_w;
        sa.Np = n_prev;
        sa.per_split = per;
        sa.st = dstate;
        sa.partial = static_cast<double*>(part);
        hipLaunchKernelGGL(k_smc_sums, dim3(bx, splits), dim3(SUMS_BLOCK), 0, s, sa);
        if ((rc = check_launch("k_smc_sums"))) return rc;
        hipLaunchKernelGGL(k_smc_finish, dim3(1), dim3(1024), 0, s, sa.partial, splits, N, w, dess);
        if ((rc = check_launch("k_smc_finish"))) return rc;
    }
    unsigned long long inbox = 0;
    double ess = 0.0;
    ABC_HIP(hipMemcpyAsync(&inbox, dbox, sizeof inbox, hipMemcpyDeviceToHost, s));
    ABC_HIP(hipMemcpyAsync(&ess, dess, sizeof ess, hipMemcpyDeviceToHost, s));
    if ((rc = sync(s))) return rc;
    stats->eps = eps;
    stats->pad = 0;
    stats->samples = samples;
    stats->in_support = gen == 0 ? samples : (int64_t)inbox;
    stats->proposed = proposed;
    stats->ess = ess;
    return ABC_OK;
}

extern "C" abc_status abc_smc_run(const abc_series* ser, const abc_model* model,
                                  const abc_prior* prior, uint64_t seed, uint32_t series,
                                  const abc_smc_config* cfg, int64_t* idx, float* theta, double* w,
                                  double* dist, abc_smc_gen_stats* stats, int32_t* gens_done,
                                  void* stream)
{
    abc_status rc;
    if ((rc = check_cfg(cfg))) return rc;
    ABC_REQUIRE(gens_done != nullptr && stats != nullptr, "NULL output");
    *gens_done = 0;
    const int N = cfg->n_particles;
    abc_smc_config c = *cfg;
    for (int t = 0; t < cfg->generations; ++t) {
        if (t > 0 && cfg->eps_min > 0.0f && stats[t - 1].eps <= cfg->eps_min) break;
        if (t > 1) {
            // first chunk sized from the previous generation's consumption (the
            // chunk schedule never changes the population, only the number of
            // round trips)
            const int64_t want = stats[t - 1].samples + stats[t - 1].samples / 4;
            int64_t c0 = cfg->chunk0;
            while (c0 < want && c0 < cfg->chunk_max) c0 <<= 1;
            c.chunk0 = c0 < cfg->chunk_max ? c0 : cfg->chunk_max;
        }
        const size_t o = (size_t)t * N, op = (size_t)(t - 1) * N;
        rc = abc_smc_generation(ser, model, prior, seed, series, t,
                                t ? theta + 8 * op : nullptr, t ? w + op : nullptr,
                                t ? dist + op : nullptr, t ? N : 0, &c, idx + o, theta + 8 * o,
                                w + o, dist + o, stats + t, nullptr, stream);
        if (rc) return rc;
        *gens_done = t + 1;
    }
    return ABC_OK;
}
