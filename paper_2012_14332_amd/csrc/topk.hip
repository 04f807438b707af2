// Nearest-k selection: the k samples with the smallest distances, ties to the
// lower sample index, returned in index order (the "keep the k nearest prior
// samples" rule of the single-country workload; the per-run Top-k return of
// Sec. 3.2), and its C-ABI entry points abc_nearest_k (float32 distances of a
// launch) and abc_nearest_k_rows (float64 distances of a small row set).
//
// abc_nearest_k never sorts the n distances. Distances map to order-preserving
// 32-bit keys; then
//   k_nk_minmax   min / max key of the distances below +inf and their count;
//   k_nk_hist     4096 linear bins over a key range (or, for a run of equal
//                 keys, over the sample index), wavefront-private LDS counts;
//                 the host narrows the range to the bin holding the k-th key
//                 until at most NK_CAP samples lie at or below the threshold
//                 (each pass shrinks the range 4096-fold);
//   k_nk_collect  composite keys (key << 32 | index) of those samples;
//   k_nk_finish   one workgroup sorts them in LDS (bitonic), keeps the first
//                 k, re-sorts those by index and writes the rows.
// Each pass reads the distances once (4 B per sample); the host synchronises
// once per pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "model.hpp"

namespace abc {

constexpr int NK_BINS = 4096;
constexpr int NK_CAP = 16384;
constexpr int NK_MAX_K = 4096;
constexpr int NK_GRID = 1024;

// IEEE order as unsigned order; -0 maps to +0 (they compare equal) and every
// NaN to the largest key, above +inf.
__device__ __forceinline__ uint32_t order_key(float d)
{
    uint32_t u = __float_as_uint(d);
    if (d != d) return 0xFFFFFFFFu;
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr uint32_t KEY_POS_INF = 0xFF800000u;  // order_key(+inf)

struct NkCtl {
    uint32_t kmin, kmax;
    unsigned long long finite;
    uint32_t count;  // collected rows
    uint32_t pad;
    uint32_t hist[NK_BINS];
};

__global__ __launch_bounds__(256) void k_nk_init(NkCtl* c)
{
    for (int b = threadIdx.x; b < NK_BINS; b += blockDim.x) c->hist[b] = 0u;
    if (threadIdx.x == 0) {
        c->kmin = 0xFFFFFFFFu;
        c->kmax = 0u;
        c->finite = 0ull;
        c->count = 0u;
    }
}

__global__ __launch_bounds__(256) void k_nk_minmax(const float* dist, int64_t n, NkCtl* c)
{
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    uint64_t cnt = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = order_key(dist[k]);
        if (key < KEY_POS_INF) {  // below +inf (NaN and +inf excluded)
            mn = min(mn, key);
            mx = max(mx, key);
            ++cnt;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, 64));
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
        cnt += __shfl_xor(cnt, off, 64);
    }
    // one set of device atomics per workgroup: the same three addresses from
    // every wavefront serialise
    __shared__ uint32_t smn[4], smx[4];
    __shared__ uint64_t scnt[4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smn[wv] = mn;
        smx[wv] = mx;
        scnt[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            mn = min(mn, smn[w]);
            mx = max(mx, smx[w]);
            cnt += scnt[w];
        }
        if (cnt) {
            atomicMin(&c->kmin, mn);
            atomicMax(&c->kmax, mx);
            atomicAdd(&c->finite, (unsigned long long)cnt);
        }
    }
}

// mode 0: keys in [lo, hi], bin = (key - lo) / width;
// mode 1: key == tie and index in [lo, hi], bin = (index - lo) / width.
struct HistArgs {
    const float* dist;
    int64_t n;
    int32_t mode;
    uint32_t tie;
    uint64_t lo, hi, width;
    NkCtl* c;
};

__global__ __launch_bounds__(256) void k_nk_hist(HistArgs a)
{
    __shared__ uint32_t h[4][NK_BINS];  // one histogram per wavefront
    const int wv = threadIdx.x >> 6;
    for (int b = threadIdx.x; b < 4 * NK_BINS; b += blockDim.x) (&h[0][0])[b] = 0u;
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = order_key(a.dist[k]);
        uint64_t v;
        bool in;
        if (a.mode == 0) {
            v = key;
            in = v >= a.lo && v <= a.hi;
        } else {
            v = (uint64_t)k;
            in = key == a.tie && v >= a.lo && v <= a.hi;
        }
        if (in) atomicAdd(&h[wv][(int)((v - a.lo) / a.width)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NK_BINS; b += blockDim.x) {
        const uint32_t s = h[0][b] + h[1][b] + h[2][b] + h[3][b];
        if (s) atomicAdd(&a.c->hist[b], s);
    }
}

__global__ __launch_bounds__(256) void k_nk_clear_hist(NkCtl* c)
{
    for (int b = threadIdx.x; b < NK_BINS; b += blockDim.x) c->hist[b] = 0u;
}

// rows with key < tkey, or key == tkey and index <= tidx
__global__ __launch_bounds__(256) void k_nk_collect(const float* dist, int64_t n, uint32_t tkey,
                                                    uint64_t tidx, NkCtl* c, uint64_t* out)
{
    const int lane = threadIdx.x & 63;
    for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < n; k0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = k0 + threadIdx.x;
        uint32_t key = 0xFFFFFFFFu;
        bool sel = false;
        if (k < n) {
            key = order_key(dist[k]);
            sel = key < tkey || (key == tkey && (uint64_t)k <= tidx);
        }
        const uint64_t m = __ballot(sel);
        if (m == 0ull) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&c->count, (uint32_t)__popcll(m));
        base = (uint32_t)__shfl((int)base, 0, 64);
        if (sel) {
            const uint32_t r = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (r < (uint32_t)NK_CAP) out[r] = ((uint64_t)key << 32) | (uint64_t)k;
        }
    }
}

__device__ void bitonic_u64(uint64_t* v, int npow)
{
    for (int k = 2; k <= npow; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < npow; t += blockDim.x) {
                const int p = t ^ j;
                if (p > t) {
                    const bool up = (t & k) == 0;
                    const uint64_t x = v[t], y = v[p];
                    if ((x > y) == up) {
                        v[t] = y;
                        v[p] = x;
                    }
                }
            }
            __syncthreads();
        }
}

struct FinishArgs {
    const uint64_t* cand;
    const NkCtl* c;
    int32_t k;
    const float* dist;
    const float* theta;  // or null: re-draw from the prior
    float lo[8], width[8];
    Key key;
    uint32_t domain, series;
    uint64_t first;
    int64_t* out_idx;
    float* out_theta;
    float* out_dist;
    float* out_kth;
};

__device__ __forceinline__ float key_to_float(uint32_t key)
{
    return __uint_as_float((key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key);
}

__global__ __launch_bounds__(1024) void k_nk_finish(FinishArgs a)
{
    extern __shared__ uint64_t v[];  // [NK_CAP]
    const int cnt = (int)min(a.c->count, (uint32_t)NK_CAP);
    int npow = 1;
    while (npow < cnt) npow <<= 1;
    for (int t = threadIdx.x; t < npow; t += blockDim.x) v[t] = t < cnt ? a.cand[t] : ~0ull;
    __syncthreads();
    bitonic_u64(v, npow);
    if (threadIdx.x == 0 && a.out_kth) *a.out_kth = key_to_float((uint32_t)(v[a.k - 1] >> 32));
    // the first k by (key, index); now order them by index
    int kpow = 1;
    while (kpow < a.k) kpow <<= 1;
    uint64_t mine[4];
    int nm = 0;
    for (int t = threadIdx.x; t < kpow; t += blockDim.x) mine[nm++] = t < a.k ? (v[t] & 0xFFFFFFFFull) : ~0ull;
    __syncthreads();
    nm = 0;
    for (int t = threadIdx.x; t < kpow; t += blockDim.x) v[t] = mine[nm++];
    __syncthreads();
    bitonic_u64(v, kpow);
    for (int r = threadIdx.x; r < a.k; r += blockDim.x) {
        const int64_t loc = (int64_t)v[r];
        const uint64_t i = a.first + (uint64_t)loc;
        a.out_idx[r] = (int64_t)i;
        if (a.out_dist) a.out_dist[r] = a.dist[loc];
        if (a.out_theta) {
            float th[8];
            if (a.theta) {
#pragma unroll
                for (int j = 0; j < 8; ++j) th[j] = a.theta[8 * loc + j];
            } else {
                prior_draw(a.key, i, a.series, a.domain, a.lo, a.width, th);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) a.out_theta[8 * r + j] = th[j];
        }
    }
}

// ---------------------------------------------------------------------------
// small row sets in float64: rank by (distance, index) in O(n^2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool row_less(double da, int64_t ia, double db, int64_t ib)
{
    // NaN sorts after every number
    const bool na = da != da, nb = db != db;
    if (na != nb) return nb;
    if (!na && da != db) return da < db;
    return ia < ib;
}

__global__ __launch_bounds__(256) void k_rows_rank(const double* d, const int64_t* idx, int64_t n,
                                                   int32_t k, int32_t* rank)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double dq = d[q];
    const int64_t iq = idx[q];
    // eight rows' loads in flight at a time (a short row set is latency-bound)
    int64_t r = 0, j = 0;
    for (; j + 8 <= n; j += 8) {
        double dj[8];
        int64_t ij[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dj[u] = d[j + u];
            ij[u] = idx[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) r += row_less(dj[u], ij[u], dq, iq) ? 1 : 0;
    }
    for (; j < n; ++j) r += row_less(d[j], idx[j], dq, iq) ? 1 : 0;
    rank[q] = r < k ? (int32_t)r : -1;
}

__global__ __launch_bounds__(256) void k_rows_place(const double* d, const int64_t* idx,
                                                    const float* theta, int64_t n, const int32_t* rank,
                                                    int64_t* out_idx, float* out_theta, double* out_d)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n || rank[q] < 0) return;
    const int64_t iq = idx[q];
    int64_t pos = 0, j = 0;  // selected rows with a smaller sample index
    for (; j + 8 <= n; j += 8) {
        int32_t rj[8];
        int64_t ij[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            rj[u] = rank[j + u];
            ij[u] = idx[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            pos += (rj[u] >= 0 && (ij[u] < iq || (ij[u] == iq && j + u < q))) ? 1 : 0;
    }
    for (; j < n; ++j) pos += (rank[j] >= 0 && (idx[j] < iq || (idx[j] == iq && j < q))) ? 1 : 0;
    out_idx[pos] = iq;
    if (out_d) out_d[pos] = d[q];
    if (out_theta)
        for (int j = 0; j < 8; ++j) out_theta[8 * pos + j] = theta[8 * q + j];
}

// workgroups of the grid-stride passes: about 16 samples per thread, so a
// short input does not pay for hundreds of LDS histogram clears and merges
static unsigned nk_grid(int64_t n)
{
    const int64_t g = (n + 4095) / 4096;
    return (unsigned)(g < NK_GRID ? (g > 0 ? g : 1) : NK_GRID);
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_nearest_k(const float* dist, const float* theta, const abc_prior* prior,
                                    const abc_stream* st, int64_t n, uint64_t first, int32_t k,
                                    int64_t* out_idx, float* out_theta, float* out_dist,
                                    float* out_kth, void* stream)
{
    ABC_REQUIRE(dist && out_idx, "dist/out_idx NULL");
    ABC_REQUIRE(n >= 1 && n < ((int64_t)1 << 32), "n must be in [1, 2^32)");
    ABC_REQUIRE(k >= 1 && k <= NK_MAX_K && k <= n, "k must be in [1, min(n, %d)]", NK_MAX_K);
    FinishArgs fa{};
    if (out_theta && !theta) {
        abc_status rc = prior_lo_width(prior, fa.lo, fa.width);
        if (rc) return rc;
        if ((rc = check_stream_sel(st))) return rc;
        fa.key = make_key(st->seed);
        fa.domain = st->domain;
        fa.series = st->series;
    }
    const hipStream_t s = as_stream(stream);
    void* mem = nullptr;
    const size_t ctl_bytes = (sizeof(NkCtl) + 255) & ~(size_t)255;
    {
        const abc_status rs = stream_scratch(s, ctl_bytes + sizeof(uint64_t) * NK_CAP, &mem);
        if (rs) return rs;
    }
    NkCtl* dc = static_cast<NkCtl*>(mem);
    uint64_t* cand = reinterpret_cast<uint64_t*>(static_cast<char*>(mem) + ctl_bytes);
    const unsigned grid = nk_grid(n);
    hipLaunchKernelGGL(k_nk_init, dim3(1), dim3(256), 0, s, dc);
    hipLaunchKernelGGL(k_nk_minmax, dim3(grid), dim3(256), 0, s, dist, n, dc);
    abc_status rc = check_launch("k_nk_minmax");
    if (rc) return rc;
    struct {
        uint32_t kmin, kmax;
        unsigned long long finite;
    } mm{};
    ABC_HIP(hipMemcpyAsync(&mm, dc, sizeof mm, hipMemcpyDeviceToHost, s));
    ABC_HIP(hipStreamSynchronize(s));
    if (mm.finite < (unsigned long long)k)
        return set_error(ABC_EINVAL, "only %llu of the %lld distances are finite, fewer than k = %d",
                         mm.finite, (long long)n, k);

    // narrow [lo, hi] on the key until the rows at or below the threshold fit
    uint32_t tkey = mm.kmax;
    uint64_t tidx = UINT64_MAX;
    uint64_t below = 0;  // rows strictly below the current range
    uint64_t lo = mm.kmin, hi = mm.kmax;
    uint32_t hist[NK_BINS];
    int mode = 0;
    uint32_t tie = 0;
    bool fits = false;
    for (int pass = 0; pass < 16 && !fits; ++pass) {
        const uint64_t span = hi - lo + 1;
        const uint64_t width = (span + NK_BINS - 1) / NK_BINS;
        HistArgs ha{dist, n, mode, tie, lo, hi, width, dc};
        hipLaunchKernelGGL(k_nk_clear_hist, dim3(1), dim3(256), 0, s, dc);
        hipLaunchKernelGGL(k_nk_hist, dim3(grid), dim3(256), 0, s, ha);
        if ((rc = check_launch("k_nk_hist"))) return rc;
        ABC_HIP(hipMemcpyAsync(hist, dc->hist, sizeof hist, hipMemcpyDeviceToHost, s));
        ABC_HIP(hipStreamSynchronize(s));
        uint64_t cum = below;
        int b = 0;
        for (; b < NK_BINS; ++b) {
            if (cum + hist[b] >= (uint64_t)k) break;
            cum += hist[b];
        }
        if (b == NK_BINS) return set_error(ABC_EHIP, "nearest-k: histogram lost rows");
        const uint64_t blo = lo + (uint64_t)b * width;
        const uint64_t bhi = blo + width - 1 < hi ? blo + width - 1 : hi;
        const uint64_t at_or_below = cum + hist[b];
        if (mode == 0) {
            tkey = (uint32_t)bhi;
            tidx = UINT64_MAX;
        } else {
            tkey = tie;
            tidx = bhi;
        }
        if (at_or_below <= (uint64_t)NK_CAP) {
            fits = true;
            break;
        }
        below = cum;
        if (width == 1 && mode == 0) {
            // a run of equal keys: continue on the sample index
            mode = 1;
            tie = (uint32_t)blo;
            lo = 0;
            hi = (uint64_t)n - 1;
        } else if (width == 1) {
            return set_error(ABC_EHIP, "nearest-k: index refinement did not converge");
        } else {
            lo = blo;
            hi = bhi;
        }
    }
    if (!fits) return set_error(ABC_EHIP, "nearest-k: threshold search did not converge");
    hipLaunchKernelGGL(k_nk_collect, dim3(grid), dim3(256), 0, s, dist, n, tkey, tidx, dc, cand);
    if ((rc = check_launch("k_nk_collect"))) return rc;
    fa.cand = cand;
    fa.c = dc;
    fa.k = k;
    fa.dist = dist;
    fa.theta = theta;
    fa.first = first;
    fa.out_idx = out_idx;
    fa.out_theta = out_theta;
    fa.out_dist = out_dist;
    fa.out_kth = out_kth;
    hipLaunchKernelGGL(k_nk_finish, dim3(1), dim3(1024), sizeof(uint64_t) * NK_CAP, s, fa);
    return check_launch("k_nk_finish");
}

extern "C" abc_status abc_nearest_k_rows(const double* dist64, const int64_t* idx, const float* theta,
                                         int64_t n, int32_t k, int64_t* out_idx, float* out_theta,
                                         double* out_dist, void* stream)
{
    ABC_REQUIRE(dist64 && idx && out_idx, "dist64/idx/out_idx NULL");
    ABC_REQUIRE(!out_theta || theta, "out_theta needs theta");
    ABC_REQUIRE(n >= 1 && n <= 65536, "n must be in [1, 65536]");
    ABC_REQUIRE(k >= 1 && k <= n, "k must be in [1, n]");
    const hipStream_t s = as_stream(stream);
    void* mem = nullptr;
    {
        const abc_status rs = stream_scratch(s, sizeof(int32_t) * (size_t)n, &mem);
        if (rs) return rs;
    }
    int32_t* rank = static_cast<int32_t*>(mem);
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    hipLaunchKernelGGL(k_rows_rank, g, b, 0, s, dist64, idx, n, k, rank);
    abc_status rc = check_launch("k_rows_rank");
    if (rc) return rc;
    hipLaunchKernelGGL(k_rows_place, g, b, 0, s, dist64, idx, theta, n, rank, out_idx, out_theta,
                       out_dist);
    return check_launch("k_rows_place");
}
