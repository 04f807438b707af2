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

#include <mutex>

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
        for (int q = 0; q < CT_STEPS; ++q) v[q] = load_stream(p + 64 * q);
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

// ---------------------------------------------------------------------------
// Two-pass compaction (abc_accept_compact). Each wavefront owns a unit of
// consecutive samples (16 steps of 4096; fewer below CP_STEP_EMIT samples). Pass 1 streams the unit's distances once and,
// with no dependency on any other wavefront, counts its accepted samples and
// keeps the unit offsets of the first CP_SLOTS of them in sample order. A
// single workgroup then forms the exclusive prefix of the unit counts, and
// pass 2 writes each unit's rows at its prefix: from the kept offsets, or --
// for a unit holding more than CP_SLOTS accepts -- by streaming the unit
// again. Rows come out in sample-index order, exactly as from the look-back
// kernel above; the streaming pass has no ticket and no look-back to wait on.
// ---------------------------------------------------------------------------
constexpr int CP_CHUNKS = 16;                        // 4096-sample steps per unit
constexpr int CP_SLOTS = 64;                         // accepted offsets kept per unit
constexpr int CP_WAVES = 4;                          // wavefronts per workgroup
// Below this many samples the units shrink to about 256 per input (down to
// one step), so that a short input spreads over many wavefronts instead of a
// few walking 16 steps each, and pass 1 also keeps each step's count so that
// pass 2 runs one wavefront per step: a unit with more accepts than kept
// offsets is then written by all its steps at once instead of one wavefront
// streaming it again (high acceptance, as in the SMC generations). Larger
// inputs keep 16-step units and one emit wavefront per unit, as most extra
// wavefronts would find nothing. The order of the rows does not depend on
// either choice.
constexpr int64_t CP_STEP_EMIT = (int64_t)1 << 22;

struct CpArgs {
    CompactArgs a;
    int32_t chunks;  // 4096-sample steps per unit
    int64_t span;    // samples per unit (CT_WAVE_SPAN chunks)
    int64_t units;
    uint32_t* cnt;   // [units]
    uint32_t* slot;  // [units][CP_SLOTS]
    int64_t* pref;   // [units]
    uint32_t* scnt;  // [units][chunks] accepts per step, or null (one emit wavefront per unit)
};

// Accept mask of one 4096-sample step of a unit: bit 4 q + c for sample
// s0 + 256 q + 4 lane + c.
__device__ __forceinline__ uint64_t step_mask(const CompactArgs& a, int64_t s0, int lane)
{
    uint64_t bits = 0;
    if (s0 + CT_WAVE_SPAN <= a.n) {
        const float4* p = reinterpret_cast<const float4*>(a.dist + s0) + lane;
        float4 v[CT_STEPS];
#pragma unroll
        for (int q = 0; q < CT_STEPS; ++q) v[q] = load_stream(p + 64 * q);
#pragma unroll
        for (int q = 0; q < CT_STEPS; ++q) {
            const uint64_t m = (uint64_t)(v[q].x <= a.eps) | ((uint64_t)(v[q].y <= a.eps) << 1) |
                               ((uint64_t)(v[q].z <= a.eps) << 2) | ((uint64_t)(v[q].w <= a.eps) << 3);
            bits |= m << (4 * q);
        }
    } else {
        for (int q = 0; q < CT_STEPS; ++q)
            for (int c = 0; c < 4; ++c) {
                const int64_t k = s0 + 256 * q + 4 * lane + c;
                if (k < a.n && a.dist[k] <= a.eps) bits |= 1ull << (4 * q + c);
            }
    }
    return bits;
}

// Visits the accepted samples of one step in sample order: f(k, r) for the
// r-th accept of the unit (r counted from r0). Returns the step's count.
template <typename F>
__device__ __forceinline__ int step_visit(uint64_t bits, int64_t s0, int lane, int64_t r0, F f)
{
    int64_t r = r0;
    for (int q = 0; q < CT_STEPS; ++q) {
        const uint32_t m = (uint32_t)(bits >> (4 * q)) & 15u;
        if (__ballot(m != 0u) == 0ull) continue;
        const int c = __popc(m);
        const int incl = wave_incl_scan_i32(c, lane);
        int64_t rr = r + (incl - c);
        for (uint32_t mm = m; mm != 0u; mm &= mm - 1u) {
            f(s0 + 256 * q + 4 * lane + (__ffs(mm) - 1), rr);
            ++rr;
        }
        r += __builtin_amdgcn_readlane(incl, 63);
    }
    return (int)(r - r0);
}

__global__ __launch_bounds__(64 * CP_WAVES) void k_cp_count(CpArgs p)
{
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * CP_WAVES + (threadIdx.x >> 6);
    if (u >= p.units) return;
    const int64_t start = u * p.span;
    uint32_t* slot = p.slot + u * CP_SLOTS;
    int64_t total = 0;
    for (int j = 0; j < p.chunks; ++j) {
        const int64_t s0 = start + (int64_t)j * CT_WAVE_SPAN;
        if (s0 >= p.a.n) break;
        const uint64_t bits = step_mask(p.a, s0, lane);
        int c = 0;
        if (__ballot(bits != 0ull) != 0ull)
            c = step_visit(bits, s0, lane, total, [&](int64_t k, int64_t r) {
                if (r < CP_SLOTS) slot[r] = (uint32_t)(k - start);
            });
        total += c;
        if (p.scnt && lane == 0) p.scnt[u * p.chunks + j] = (uint32_t)c;
    }
    if (lane == 0) p.cnt[u] = (uint32_t)total;
}

// Exclusive prefix of the unit counts in one workgroup of 1024 threads:
// thread t sums a contiguous block of units, the block sums are scanned in
// LDS, then each thread writes its block's prefixes in order.
__global__ __launch_bounds__(1024) void k_cp_scan(CpArgs p)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (p.units + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < p.units ? b0 + per : p.units;
    int64_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += p.cnt[b];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        p.pref[b] = run;
        run += p.cnt[b];
    }
    if (t == 1023) *p.a.out_count = part[1023];
}

__global__ __launch_bounds__(64 * CP_WAVES) void k_cp_emit(CpArgs p)
{
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * CP_WAVES + (threadIdx.x >> 6);
    if (u >= p.units) return;
    const uint32_t c = p.cnt[u];
    if (c == 0) return;
    const int64_t base = p.pref[u];
    if (base >= p.a.capacity) return;
    const int64_t start = u * p.span;
    if (c <= (uint32_t)CP_SLOTS) {
        for (uint32_t j = lane; j < c; j += 64)
            emit_row(p.a, start + p.slot[u * CP_SLOTS + j], base + j);
        return;
    }
    // more accepts than kept offsets: stream the unit again, in order
    int64_t total = 0;
    for (int j = 0; j < p.chunks; ++j) {
        const int64_t s0 = start + (int64_t)j * CT_WAVE_SPAN;
        if (s0 >= p.a.n || base + total >= p.a.capacity) break;
        const uint64_t bits = step_mask(p.a, s0, lane);
        if (__ballot(bits != 0ull) == 0ull) continue;
        total += step_visit(bits, s0, lane, total, [&](int64_t k, int64_t r) {
            emit_row(p.a, k, base + r);
        });
    }
}

// Pass 2 with one wavefront per step (inputs below CP_STEP_EMIT): a unit
// within its kept offsets is written by its first step's wavefront; otherwise
// each step's wavefront writes that step's accepts after those of the unit's
// earlier steps.
__global__ __launch_bounds__(64 * CP_WAVES) void k_cp_emit_steps(CpArgs p)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * CP_WAVES + (threadIdx.x >> 6);
    const int64_t u = w / p.chunks;
    const int j = (int)(w - u * p.chunks);
    if (u >= p.units) return;
    const uint32_t c = p.cnt[u];
    if (c == 0) return;
    const int64_t base = p.pref[u];
    if (base >= p.a.capacity) return;
    const int64_t start = u * p.span;
    if (c <= (uint32_t)CP_SLOTS) {
        if (j != 0) return;
        for (uint32_t q = lane; q < c; q += 64)
            emit_row(p.a, start + p.slot[u * CP_SLOTS + q], base + q);
        return;
    }
    const int64_t s0 = start + (int64_t)j * CT_WAVE_SPAN;
    if (s0 >= p.a.n) return;
    const uint32_t* sc = p.scnt + u * p.chunks;
    int64_t off = 0;
    for (int q = 0; q < j; ++q) off += sc[q];
    if (sc[j] == 0u || base + off >= p.a.capacity) return;
    const uint64_t bits = step_mask(p.a, s0, lane);
    step_visit(bits, s0, lane, 0, [&](int64_t k, int64_t r) { emit_row(p.a, k, base + off + r); });
}

}  // namespace abc

using namespace abc;

// Scratch of the allocation-free entry point: one status word per tile plus
// the ticket, for at most CT_STATIC_TILES tiles. Every GPU the library runs on
// holds its own copy until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device (the array's
// name is a host-side stand-in, not a device address).
constexpr int64_t CT_STATIC_TILES = 16384;
static __device__ __align__(256) unsigned long long scratch[CT_STATIC_TILES + 1];

namespace {

constexpr int CT_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[CT_MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
abc_status static_scratch(unsigned long long** out)
{
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    ABC_REQUIRE(dev >= 0 && dev < CT_MAX_DEVICES, "device %d beyond the library's %d", dev,
                CT_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return set_error(ABC_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = reinterpret_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[dev];
    return ABC_OK;
}

int compact_waves(int64_t n) { return n >= CT_BIG_N ? CT_WAVES_BIG : CT_WAVES_SMALL; }

int64_t compact_tiles(int64_t n)
{
    const int64_t tile = (int64_t)compact_waves(n) * CT_WAVE_SPAN;
    return (n + tile - 1) / tile;
}

// Validates the arguments and fills everything but the scratch words.
abc_status compact_args(const float* dist, const float* theta, const float* weight,
                        const abc_prior* prior, const abc_stream* st, int64_t n, uint64_t first,
                        float eps, int64_t capacity, int64_t* out_idx, float* out_theta,
                        float* out_dist, float* out_w, int64_t* out_count, CompactArgs& a)
{
    ABC_REQUIRE(n >= 0 && capacity >= 0, "n and capacity must be >= 0");
    ABC_REQUIRE(out_count != nullptr, "out_count is NULL");
    ABC_REQUIRE(!isnan(eps), "eps is NaN");
    a = CompactArgs{};
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
    a.num_tiles = compact_tiles(n);
    return ABC_OK;
}

// Enqueues the clearing kernel and the compaction on `s`; `words` holds
// num_tiles + 1 device words (status words, then the ticket).
abc_status compact_launch(CompactArgs& a, unsigned long long* words, hipStream_t s)
{
    a.status = words;
    a.ticket = reinterpret_cast<unsigned int*>(words + a.num_tiles);
    const int64_t init_n = a.num_tiles > 0 ? a.num_tiles : 1;
    hipLaunchKernelGGL(k_compact_init, dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0, s,
                       a.status, a.num_tiles, a.ticket, a.out_count);
    abc_status rc = check_launch("k_compact_init");
    if (rc == ABC_OK && a.num_tiles > 0) {
        if (compact_waves(a.n) == CT_WAVES_BIG)
            hipLaunchKernelGGL((k_compact<CT_WAVES_BIG>), dim3((unsigned)a.num_tiles),
                               dim3(64 * CT_WAVES_BIG), 0, s, a);
        else
            hipLaunchKernelGGL((k_compact<CT_WAVES_SMALL>), dim3((unsigned)a.num_tiles),
                               dim3(64 * CT_WAVES_SMALL), 0, s, a);
        rc = check_launch("k_compact");
    }
    return rc;
}

}  // namespace

extern "C" abc_status abc_accept_compact(const float* dist, const float* theta,
                                         const float* weight, const abc_prior* prior,
                                         const abc_stream* st, int64_t n, uint64_t first,
                                         float eps, int64_t capacity, int64_t* out_idx,
                                         float* out_theta, float* out_dist, float* out_w,
                                         int64_t* out_count, void* stream)
{
    CompactArgs a;
    abc_status rc = compact_args(dist, theta, weight, prior, st, n, first, eps, capacity, out_idx,
                                 out_theta, out_dist, out_w, out_count, a);
    if (rc) return rc;
    const hipStream_t s = as_stream(stream);
    // two passes; scratch (unit counts, kept offsets, prefixes) from the
    // stream's buffer
    CpArgs p{};
    p.a = a;
    p.chunks = CP_CHUNKS;
    if (n < CP_STEP_EMIT) {
        const int64_t c = (n + CT_WAVE_SPAN * 256 - 1) / (CT_WAVE_SPAN * 256);  // about 256 units
        p.chunks = c < 1 ? 1 : (int32_t)c;
    }
    p.span = (int64_t)CT_WAVE_SPAN * p.chunks;
    p.units = (n + p.span - 1) / p.span;
    const int64_t units = p.units > 0 ? p.units : 1;
    const bool steps = n < CP_STEP_EMIT;
    void* mem = nullptr;
    const size_t bytes = sizeof(int64_t) * (size_t)units + sizeof(uint32_t) * (size_t)units +
                         sizeof(uint32_t) * (size_t)CP_SLOTS * (size_t)units +
                         (steps ? sizeof(uint32_t) * (size_t)p.chunks * (size_t)units : 0);
    if ((rc = stream_scratch(s, bytes, &mem))) return rc;
    p.pref = static_cast<int64_t*>(mem);
    p.cnt = reinterpret_cast<uint32_t*>(p.pref + units);
    p.slot = p.cnt + units;
    p.scnt = steps ? p.slot + (size_t)CP_SLOTS * (size_t)units : nullptr;
    const unsigned grid = (unsigned)((units + CP_WAVES - 1) / CP_WAVES);
    if (p.units > 0) {
        hipLaunchKernelGGL(k_cp_count, dim3(grid), dim3(64 * CP_WAVES), 0, s, p);
        if ((rc = check_launch("k_cp_count"))) return rc;
    }
    hipLaunchKernelGGL(k_cp_scan, dim3(1), dim3(1024), 0, s, p);  // also writes the count
    if ((rc = check_launch("k_cp_scan"))) return rc;
    if (p.units > 0 && capacity > 0) {
        if (steps) {
            const int64_t waves = p.units * p.chunks;
            hipLaunchKernelGGL(k_cp_emit_steps, dim3((unsigned)((waves + CP_WAVES - 1) / CP_WAVES)),
                               dim3(64 * CP_WAVES), 0, s, p);
            rc = check_launch("k_cp_emit_steps");
        } else {
            hipLaunchKernelGGL(k_cp_emit, dim3(grid), dim3(64 * CP_WAVES), 0, s, p);
            rc = check_launch("k_cp_emit");
        }
    }
    return rc;
}

extern "C" abc_status abc_accept_compact_noalloc(const float* dist, const float* theta,
                                                 const float* weight, const abc_prior* prior,
                                                 const abc_stream* st, int64_t n, uint64_t first,
                                                 float eps, int64_t capacity, int64_t* out_idx,
                                                 float* out_theta, float* out_dist, float* out_w,
                                                 int64_t* out_count, void* stream)
{
    ABC_REQUIRE(n <= ABC_NOALLOC_COMPACT_MAX_N, "n = %lld exceeds ABC_NOALLOC_COMPACT_MAX_N = %lld",
                (long long)n, (long long)ABC_NOALLOC_COMPACT_MAX_N);
    CompactArgs a;
    abc_status rc = compact_args(dist, theta, weight, prior, st, n, first, eps, capacity, out_idx,
                                 out_theta, out_dist, out_w, out_count, a);
    if (rc) return rc;
    if (a.num_tiles > CT_STATIC_TILES)  // cannot happen below the size limit; kept as a guard
        return set_error(ABC_EINVAL, "%lld tiles exceed the static scratch of %lld",
                         (long long)a.num_tiles, (long long)CT_STATIC_TILES);
    unsigned long long* words = nullptr;
    if ((rc = static_scratch(&words))) return rc;
    return compact_launch(a, words, as_stream(stream));
}
