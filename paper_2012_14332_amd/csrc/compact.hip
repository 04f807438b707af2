// Accept-reject and stable compaction of accepted samples (Sec. 2.2, eq. 7;
// Sec. 3.2), and its C-ABI entry point abc_accept_compact.
//
// Single pass over the distances with a decoupled look-back scan: every
// workgroup takes the next tile of 16384 or 65536 samples from an atomic ticket (so a
// tile only ever waits on tiles that are already running), counts its
// accepted samples, publishes that aggregate, then one wavefront looks back
// over up to 64 predecessor tiles at a time to obtain the exclusive prefix.
// Each wavefront owns 4096 consecutive samples of the tile and reads them as
// 16 coalesced float4 loads per lane (1 KB per load instruction), keeping a
// 4-bit accept mask per load; ranks inside a load are only formed for the
// rare loads that hold an accepted sample. Output order is sample-index
// order, so the result does not depend on scheduling. HBM traffic: 4 B per
// sample read, plus 32-48 B per accepted row (theta re-drawn from its counter
// when it was never materialised). Large tiles keep the ticket counter and
// the look-back -- device-scope atomics on few addresses -- off the critical
// path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "model.hpp"

namespace abc {

constexpr int CT_STEPS = 16;                     // float4 loads per lane
constexpr int CT_WAVE_SPAN = 64 * 4 * CT_STEPS;  // 4096 samples per wavefront
// Wavefronts per workgroup (tile = WAVES x 4096 samples): 16 for large inputs,
// where fewer tickets and look-backs pay; 4 below CT_BIG_N, where small
// workgroups also fit beside a resident simulate launch on another stream.
constexpr int CT_WAVES_BIG = 16;
constexpr int CT_WAVES_SMALL = 4;
constexpr int64_t CT_BIG_N = (int64_t)1 << 25;

constexpr uint64_t ST_AGG = 1;     // status word: (value << 2) | flag
constexpr uint64_t ST_PREFIX = 2;

struct CompactArgs {
    const float* dist;
    const float* theta;
    const float* weight;
    float lo[8];
    float width[8];
    Key key;
    uint32_t domain;
    uint32_t series;
    int64_t n;
    uint64_t first;
    float eps;
    int64_t capacity;
    int64_t* out_idx;
    float* out_theta;
    float* out_dist;
    float* out_w;
    int64_t* out_count;
    unsigned long long* status;  // [num_tiles]
    unsigned int* ticket;
    int64_t num_tiles;
};

__global__ void k_compact_init(unsigned long long* status, int64_t num_tiles, unsigned int* ticket,
                               int64_t* out_count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < num_tiles) status[k] = 0ull;
    if (k == 0) {
        *ticket = 0u;
        *out_count = 0;
    }
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// One accepted sample k of the tile goes to output row r.
__device__ __forceinline__ void emit_row(const CompactArgs& a, int64_t k, int64_t r)
{
    if (r >= a.capacity) return;
    const uint64_t i = a.first + (uint64_t)k;
    a.out_idx[r] = (int64_t)i;
    float th[8];
    if (a.theta) {
#pragma unroll
        for (int j = 0; j < 8; ++j) th[j] = a.theta[8 * k + j];
    } else {
        prior_draw(a.key, i, a.series, a.domain, a.lo, a.width, th);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) a.out_theta[8 * r + j] = th[j];
    if (a.out_dist) a.out_dist[r] = a.dist[k];
    if (a.out_w) a.out_w[r] = a.weight[k];
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_compact(CompactArgs a)
{
    constexpr int CT_TILE = WAVES * CT_WAVE_SPAN;
    __shared__ unsigned int tile_sh;
    __shared__ int wave_tot[WAVES];
    __shared__ int64_t excl_sh;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0) tile_sh = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t tile = tile_sh;
    const int64_t wbase = tile * CT_TILE + (int64_t)wave * CT_WAVE_SPAN;

    // accept masks: bit 4 q + c for sample wbase + 256 q + 4 lane + c
    uint64_t bits = 0;
    if (wbase + CT_WAVE_SPAN <= a.n) {
        const float4* p = reinterpret_cast<const float4*>(a.dist + wbase) + lane;
        float4 v[CT_STEPS];
#pragma unroll
        for (int q = 0; q < CT_STEPS; ++q) v[q] = p[64 * q];
#pragma unroll
        for (int q = 0; q < CT_STEPS; ++q) {
            const uint64_t m = (uint64_t)(v[q].x <= a.eps) | ((uint64_t)(v[q].y <= a.eps) << 1) |
                               ((uint64_t)(v[q].z <= a.eps) << 2) | ((uint64_t)(v[q].w <= a.eps) << 3);
            bits |= m << (4 * q);
        }
    } else {
        for (int q = 0; q < CT_STEPS; ++q)
            for (int c = 0; c < 4; ++c) {
                const int64_t k = wbase + 256 * q + 4 * lane + c;
                if (k < a.n && a.dist[k] <= a.eps) bits |= 1ull << (4 * q + c);
            }
    }
    const int cnt = __popcll(bits);
    const int wsum = __builtin_amdgcn_readlane(wave_incl_scan_i32(cnt, lane), 63);
    if (lane == 0) wave_tot[wave] = wsum;
    __syncthreads();
    int wave_off = 0, block_tot = 0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) {
        if (q < wave) wave_off += wave_tot[q];
        block_tot += wave_tot[q];
    }

    // publish the aggregate, then look back for the exclusive prefix
    if (wave == 0) {
        int64_t excl = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&a.status[0], ((uint64_t)block_tot << 2) | ST_PREFIX,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&a.status[tile], ((uint64_t)block_tot << 2) | ST_AGG,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t look = tile - 1;
            while (true) {
                const int64_t p = look - lane;
                uint64_t st = (uint64_t)ST_PREFIX;  // before tile 0: prefix 0
                if (p >= 0)
                    st = __hip_atomic_load(&a.status[p], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = st & 3u;
                if (__ballot(flag == 0) != 0ull) continue;  // a predecessor has not published yet
                const uint64_t pm = __ballot(flag == ST_PREFIX);
                const int64_t val = (int64_t)(st >> 2);
                if (pm != 0ull) {
                    const int stop = __ffsll((unsigned long long)pm) - 1;  // nearest prefix
                    excl += wave_sum_i64(lane <= stop ? val : 0);
                    break;
                }
                excl += wave_sum_i64(val);
                look -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&a.status[tile], ((uint64_t)(excl + block_tot) << 2) | ST_PREFIX,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            excl_sh = excl;
            if (tile == a.num_tiles - 1) *a.out_count = excl + block_tot;
        }
    }
    __syncthreads();
    if (wsum == 0) return;

    // rows in sample order: load by load, lanes in order, components in order
    int64_t r0 = excl_sh + wave_off;
    for (int q = 0; q < CT_STEPS; ++q) {
        const uint32_t m = (uint32_t)(bits >> (4 * q)) & 15u;
        if (__ballot(m != 0u) == 0ull) continue;
        const int c = __popc(m);
        const int incl = wave_incl_scan_i32(c, lane);
        int64_t r = r0 + (incl - c);
        for (uint32_t mm = m; mm != 0u; mm &= mm - 1u) {
            emit_row(a, wbase + 256 * q + 4 * lane + (__ffs(mm) - 1), r);
            ++r;
        }
        r0 += __builtin_amdgcn_readlane(incl, 63);
    }
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_accept_compact(const float* dist, const float* theta,
                                         const float* weight, const abc_prior* prior,
                                         const abc_stream* st, int64_t n, uint64_t first,
                                         float eps, int64_t capacity, int64_t* out_idx,
                                         float* out_theta, float* out_dist, float* out_w,
                                         int64_t* out_count, void* stream)
{
    ABC_REQUIRE(n >= 0 && capacity >= 0, "n and capacity must be >= 0");
    ABC_REQUIRE(out_count != nullptr, "out_count is NULL");
    ABC_REQUIRE(!isnan(eps), "eps is NaN");
    CompactArgs a{};
    if (n > 0) {
        ABC_REQUIRE((weight == nullptr) == (out_w == nullptr),
                    "weight and out_w must both be set or both NULL");
        ABC_REQUIRE(dist != nullptr, "dist is NULL");
        ABC_REQUIRE((reinterpret_cast<uintptr_t>(dist) & 15u) == 0, "dist must be 16-byte aligned");
        if (capacity > 0) ABC_REQUIRE(out_idx != nullptr && out_theta != nullptr, "out_idx/out_theta NULL");
        if (theta == nullptr) {
            abc_status rc = prior_lo_width(prior, a.lo, a.width);
            if (rc) return rc;
            if ((rc = check_stream_sel(st))) return rc;
            a.key = make_key(st->seed);
            a.domain = st->domain;
            a.series = st->series;
        }
    }
    const hipStream_t s = as_stream(stream);
    const int waves = n >= CT_BIG_N ? CT_WAVES_BIG : CT_WAVES_SMALL;
    const int64_t tile = (int64_t)waves * CT_WAVE_SPAN;
    const int64_t num_tiles = (n + tile - 1) / tile;
    // scratch: one status word per tile + the ticket, stream-ordered
    void* scratch = nullptr;
    const size_t bytes = sizeof(unsigned long long) * (size_t)(num_tiles + 1);
    ABC_HIP(hipMallocAsync(&scratch, bytes, s));
    a.status = reinterpret_cast<unsigned long long*>(scratch);
    a.ticket = reinterpret_cast<unsigned int*>(a.status + num_tiles);
    a.dist = dist;
    a.theta = theta;
    a.weight = weight;
    a.n = n;
    a.first = first;
    a.eps = eps;
    a.capacity = capacity;
    a.out_idx = out_idx;
    a.out_theta = out_theta;
    a.out_dist = out_dist;
    a.out_w = out_w;
    a.out_count = out_count;
    a.num_tiles = num_tiles;
    const int64_t init_n = num_tiles > 0 ? num_tiles : 1;
    hipLaunchKernelGGL(k_compact_init, dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0, s,
                       a.status, num_tiles, a.ticket, out_count);
    abc_status rc = check_launch("k_compact_init");
    if (rc == ABC_OK && num_tiles > 0) {
        if (waves == CT_WAVES_BIG)
            hipLaunchKernelGGL((k_compact<CT_WAVES_BIG>), dim3((unsigned)num_tiles),
                               dim3(64 * CT_WAVES_BIG), 0, s, a);
        else
            hipLaunchKernelGGL((k_compact<CT_WAVES_SMALL>), dim3((unsigned)num_tiles),
                               dim3(64 * CT_WAVES_SMALL), 0, s, a);
        rc = check_launch("k_compact");
    }
    hipError_t e = hipFreeAsync(scratch, s);
    if (rc == ABC_OK && e != hipSuccess) return set_error(ABC_EHIP, "hipFreeAsync: %s", hipGetErrorString(e));
    return rc;
}
