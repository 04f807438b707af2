// Prior sampling, simulate+distance and trajectory recording kernels, and their
// C-ABI entry points (abc_sample_prior, abc_simulate_distance,
// abc_simulate_record).
//
// simulate+distance: one lane per trajectory. The observed series of the
// launch is staged once per workgroup in LDS as log1p(O) (or O for the raw
// distance), so the day loop touches no global memory at all: per sample the
// kernel reads 32 B of theta (or none when theta is drawn in-kernel) and
// writes 4 B of distance. A sample leaves the day loop as soon as its running
// squared distance passes the early-exit bound.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bound.hpp"
#include "common.hpp"
#include "model.hpp"

namespace abc {

constexpr int SIM_BLOCK = 256;

struct SimArgs {
    const float* theta;  // [n][8] or null -> prior draw
    float lo[8];
    float width[8];
    float hi[8];         // support check of supplied theta (box != 0)
    int32_t box;
    Key key;
    uint32_t domain;
    uint32_t series;
    uint64_t first;
    int64_t n;
    int32_t P, A0, R0, D0, T;
    const int32_t* obs;  // [3][T]
    float scale;
    float exit_f32;      // squared-distance early-exit bound (float path)
    double exit_f64;     // same, double path
    float* dist;
    double* dist64;
    unsigned long long* days;  // nullable: += sample-days executed
    int32_t* traj;       // record mode: [n][T+1][6]
    int32_t refill_min;  // refill a wave's idle lanes once at least this many are idle
    int32_t lb_ntb;      // future-days bound table: time blocks (0 = no bound)
    int32_t lb_sh;       // days per time block = 2^lb_sh
};

__device__ __forceinline__ void load_or_draw_theta(const SimArgs& a, bool prior, int64_t k,
                                                   uint64_t i, float th[8])
{
    if (prior) {
        prior_draw(a.key, i, a.series, a.domain, a.lo, a.width, th);
    } else {
        const float4* p = reinterpret_cast<const float4*>(a.theta + 8 * k);
        const float4 x = p[0], y = p[1];
        th[0] = x.x; th[1] = x.y; th[2] = x.z; th[3] = x.w;
        th[4] = y.x; th[5] = y.y; th[6] = y.z; th[7] = y.w;
    }
}

// Prior support of a supplied theta (closed box; NaN is outside).
__device__ __forceinline__ bool outside_box(const SimArgs& a, const float th[8])
{
    bool out = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) out |= !(th[j] >= a.lo[j] && th[j] <= a.hi[j]);
    return out;
}

// ---------------------------------------------------------------------------
// float32 simulate + distance with per-wave lane refill
//
// Each wavefront owns a fixed set of 64-sample chunks (chunk c = wave id +
// j * number of waves) and walks through them as a queue. A lane whose
// sample is finished -- early exit or day T reached -- writes its distance
// and takes the next queue position at once, so lanes never idle behind the
// slowest trajectory of the wave. Per-sample constants (rates, I0) are
// produced 64 at a time by the whole wave into a small per-wave LDS ring,
// which keeps the prior draw (two Philox calls) out of the divergent refill
// branch. SPL independent sample slots per lane add instruction-level
// parallelism. The result of each sample depends only on its index and
// theta, never on the launch shape or on which lane ran it.
// ---------------------------------------------------------------------------
// Everything a lane needs to start a sample, prepared by the whole wave so the
// divergent refill branch only copies 64 bytes out of LDS.
struct alignas(16) Slot {
    float a0, al, n, be, ga, de, bh;
    int32_t i0;
    uint32_t c1base, g3, h3, f3;  // per-sample part of Philox rounds 1-3
    int64_t k;                    // sample offset in the launch (n = no sample)
    int64_t pad;
};

template <bool PRIOR>
__device__ __forceinline__ void fill_slot(const SimArgs& a, int64_t k, uint32_t u0, Slot& out)
{
    float thv[8];
    load_or_draw_theta(a, PRIOR, k, a.first + (uint64_t)k, thv);
    const Theta th = theta_from(thv);
    const RatesF r = rates_f32(th);
    const State s0 = init_state(th.ka, a.P, a.A0, a.R0, a.D0);
    PhiloxDays ph;
    ph.begin(a.first + (uint64_t)k, u0, a.key);
    out.a0 = r.a0; out.al = r.al; out.n = r.n; out.be = r.be;
    out.ga = r.ga; out.de = r.de; out.bh = r.bh; out.i0 = s0.I;
    out.c1base = ph.c1base; out.g3 = ph.g3; out.h3 = ph.h3; out.f3 = ph.f3;
    out.k = k;
    out.pad = (!PRIOR && a.box && outside_box(a, thv)) ? 1 : 0;  // 1: prior density zero
}

struct Lane {
    State s;
    RatesF r;
    PhiloxDays ph;
    int64_t k;     // sample offset within the launch
    int32_t t;     // next day to simulate; 0: no sample (idle)
    float acc, comp;
};

template <int NOISE, int DIST, bool KAHAN, bool PRIOR, int SPL>
__global__ __launch_bounds__(1024 / SPL) void k_simulate_f32(SimArgs a)
{
    constexpr int RING = 64;  // one chunk of 64 queue positions
    extern __shared__ float lds_f[];
    const int T = a.T;
    const int obs_words = (3 * T + 3) & ~3;
    const int ntb = DIST == 0 ? a.lb_ntb : 0;
    float* tab = lds_f + obs_words;  // [2][ntb][LB_Q] future-days bound
    Slot* ring_all = reinterpret_cast<Slot*>(lds_f + obs_words + 2 * LB_Q * ntb);

    // observed series: log2(1 + O) for the log1p distance (accumulated in
    // log2 units), or the count itself for the raw distance
    for (int q = threadIdx.x; q < 3 * T; q += blockDim.x) {
        const int32_t O = a.obs[q];
        if (DIST == 0)
            lds_f[q] = (float)(log1p((double)O) * 1.44269504088896340736);
        else
            lds_f[q] = __int_as_float(O);
    }
    if (DIST == 0 && ntb > 0) {
        // b_s of R and D in float64, staged where the ring will live
        double* stage = reinterpret_cast<double*>(ring_all);
        for (int q = threadIdx.x; q < 2 * T; q += blockDim.x)
            stage[q] = log1p((double)a.obs[T + q]) * 1.44269504088896340736;
        __syncthreads();
        build_future_bound(stage, T, a.lb_sh, ntb, (double)a.exit_f32, tab);
    }
    __syncthreads();

    // The float32 waves take issue priority over waves of other kernels
    // sharing the compute unit (the float64 band decision of the previous
    // launch runs beside this one and fills the gaps instead of holding up
    // the waves whose static share of the launch it would delay).
    __builtin_amdgcn_s_setprio(1);
    const int lane = threadIdx.x & 63;
    // the wavefront index is uniform over the wave: kept scalar, so is the
    // queue arithmetic derived from it
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Slot* ring = ring_all + wv * RING;
    const int64_t wg = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nchunks = (a.n + 63) >> 6;
    if (wg >= nchunks) return;
    // queue positions of this wave (fits 32 bits: the host limits n per launch);
    // its j-th chunk is wg + j nw
    const uint32_t Q = (uint32_t)(((nchunks - 1 - wg) / nw + 1) << 6);

    const PhiloxSeries ps = philox_series(a.series, a.key);
    const float invP = 1.0f / (float)a.P;
    const float nc = noise_c(a.scale);
    const float dscale = DIST == 0 ? 0.693147180559945309417f : 1.0f;
    const uint32_t wdom = a.domain << 4;

    // the ring holds one chunk: sample offsets 64 c + lane
    auto fill = [&](int64_t c) {
        const int64_t k = (c << 6) + lane;
        Slot& sl = ring[lane];
        if (k < a.n)
            fill_slot<PRIOR>(a, k, ps.u0, sl);
        else
            sl.k = a.n;
    };

    // wave-uniform queue state, kept in scalar registers
    uint32_t qb = 0;               // next queue position
    uint32_t filled = 0xFFFFFFFFu; // chunk currently in the ring
    Lane L[SPL];
#pragma unroll
    for (int j = 0; j < SPL; ++j) L[j].t = 0;
    uint32_t days_done = 0;

    while (true) {
        // refill every idle slot from the wave queue, in queue order; a refill
        // may span the end of one chunk and the start of the next
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
            uint64_t m = __ballot(L[j].t == 0);
            if (__popcll(m) < a.refill_min) continue;  // let a few more lanes finish first
            while (m != 0ull && qb < Q) {
                const uint32_t jc = qb >> 6;
                if (jc != filled) {
                    fill(wg + (int64_t)jc * nw);
                    filled = jc;
                }
                const uint32_t avail = 64u - (qb & 63u);
                const bool inm = (m >> lane) & 1ull;
                // lanes of m below this one
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const bool take = inm && rank < avail;
                if (take) {
                    const Slot sl = ring[(qb & 63u) + rank];
                    if (!PRIOR && sl.k < a.n && sl.pad != 0) {
                        a.dist[sl.k] = INFINITY;
                        if (a.dist64) a.dist64[sl.k] = (double)INFINITY;
                    } else if (sl.k < a.n) {
                        Lane& l = L[j];
                        l.r = RatesF{sl.a0, sl.al, sl.n, sl.be, sl.ga, sl.de, sl.bh};
                        l.s.A = a.A0; l.s.R = a.R0; l.s.D = a.D0; l.s.Ru = 0;
                        l.s.I = sl.i0;
                        l.s.S = a.P - (a.A0 + a.R0 + a.D0) - sl.i0;
                        l.ph.c1base = sl.c1base; l.ph.g3 = sl.g3; l.ph.h3 = sl.h3; l.ph.f3 = sl.f3;
                        l.k = sl.k;
                        l.t = 1;
                        l.acc = 0.0f;
                        l.comp = 0.0f;
                    }
                }
                const uint32_t cnt = (uint32_t)__popcll(m);
                qb = __builtin_amdgcn_readfirstlane(qb + (cnt < avail ? cnt : avail));
                m = __ballot(inm && !take);  // lanes still without a position
            }
        }
        bool any = false;
#pragma unroll
        for (int j = 0; j < SPL; ++j) any |= L[j].t != 0;
        if (__ballot(any) == 0ull && qb >= Q) break;

        // one day of every active slot
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
            Lane& l = L[j];
            if (l.t == 0) continue;
            const int t = l.t;
            const uint4 w = l.ph.day(((uint32_t)t << 8) | wdom, ps.b1, a.key);
            Noise32 z;
            normals_f32(w, nc, z);
            day_step_f32<NOISE>(l.s, l.r, invP, z);
            const int32_t X[3] = {l.s.A, l.s.R, l.s.D};
            float lx[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float d;
                if (DIST == 0) {
                    lx[c] = log2p1_count_f32(X[c]);
                    d = lx[c] - lds_f[c * T + t - 1];
                } else {
                    d = (float)(X[c] - __float_as_int(lds_f[c * T + t - 1]));
                }
                if (KAHAN) {
                    const float y = fmaf(d, d, -l.comp);
                    const float tt = l.acc + y;
                    l.comp = (tt - l.acc) - y;
                    l.acc = tt;
                } else {
                    l.acc = fmaf(d, d, l.acc);
                }
            }
            float lb = 0.0f;
            if (DIST == 0 && ntb > 0) {
                // grid index rounded down, below the float32 error of lx
                const float* row = tab + ((t >> a.lb_sh) * LB_Q);
                const int qr = (int)fmaf(lx[1], 2.0f, -0x1p-12f);
                const int qd = (int)fmaf(lx[2], 2.0f, -0x1p-12f);
                lb = row[qr] + row[ntb * LB_Q + qd];
            }
            const bool exited = l.acc + lb > a.exit_f32;
            if (exited || t == T) {
                const float dd = exited ? INFINITY : finish_distance_f32(l.acc, dscale);
                a.dist[l.k] = dd;
                if (a.dist64) a.dist64[l.k] = (double)dd;
                l.t = 0;
                days_done += (uint32_t)t;
            } else {
                l.t = t + 1;
            }
        }
    }
    if (a.days) {
        uint64_t v = days_done;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) atomicAdd(a.days, (unsigned long long)v);
    }
}

// ---------------------------------------------------------------------------
// float64 simulate + distance (precision study, recheck of borderline samples)
// ---------------------------------------------------------------------------

template <int NOISE, int DIST, bool PRIOR>
__global__ __launch_bounds__(SIM_BLOCK) void k_simulate_f64(SimArgs a)
{
    extern __shared__ double lds_d[];  // [3][T]
    stage_obs_f64<DIST>(a.obs, a.T, lds_d);
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;
    float thv[8];
    load_or_draw_theta(a, PRIOR, k, i, thv);
    if (!PRIOR && a.box && outside_box(a, thv)) {
        a.dist[k] = INFINITY;
        if (a.dist64) a.dist64[k] = (double)INFINITY;
        return;
    }
    const double dd = simulate_one_f64<NOISE, DIST>(thv, i, a.key, a.series, a.domain, a.P, a.A0,
                                                    a.R0, a.D0, a.T, (double)a.scale, lds_d,
                                                    a.exit_f64);
    a.dist[k] = (float)dd;
    if (a.dist64) a.dist64[k] = dd;
}

// Float64 decision for the candidates of a float32 pass (compacted at
// eps (1 + w)): rows whose float32 distance lies above eps (1 - w) are
// simulated again in float64 and decided by that distance; then the kept
// rows are compacted in place, in their original order. One workgroup.
struct RecheckArgs {
    SimArgs sim;
    float eps;
    float band_lo;   // eps (1 - w)
    float band_hi;   // eps (1 + w)
    int64_t capacity;
    int64_t* idx;
    float* theta;
    float* dist;
    float* weight;
    int64_t* count;
    uint8_t* keep;   // scratch [capacity]
    int32_t* rechecked;  // nullable: number of rows simulated in float64
    int32_t rows_max;    // rows per wavefront the LDS was sized for
    int32_t scan_min;    // candidates per wavefront at least
    int32_t all_rows;    // 1: every candidate is decided in float64, not only the band
    double* dist64;      // nullable [capacity]: float64 distance of each row so decided
};

// LDS of the float64 row kernels, for up to R rows per wavefront (W = ROW_WINDOW days):
// obs [3 T] f64 | zs [R][5 W] f64 | rix [R] u64 | rq [R] i64 | rw [R] | xs [R][3 W] i32 | rth [R][8] f32
struct RowLds {
    double* lobs;
    double* zs;
    uint64_t* rix;
    int64_t* rq;
    RowWalk* rw;
    int32_t* xs;
    float* rth;
};

__device__ __forceinline__ RowLds row_lds(double* base, int T, int R)
{
    RowLds l;
    l.lobs = base;
    l.zs = base + 3 * T;
    l.rix = reinterpret_cast<uint64_t*>(l.zs + (size_t)5 * ROW_WINDOW * R);
    l.rq = reinterpret_cast<int64_t*>(l.rix + R);
    l.rw = reinterpret_cast<RowWalk*>(l.rq + R);
    l.xs = reinterpret_cast<int32_t*>(l.rw + R);
    l.rth = reinterpret_cast<float*>(l.xs + (size_t)3 * ROW_WINDOW * R);
    return l;
}

// Pass 1: each wavefront scans a contiguous block of candidates (enough for
// the grid to cover the candidate count, at least scan_min), 64 at a time;
// the in-band ones are gathered, in candidate order, into groups of up to
// rows_max rows that are simulated side by side in float64
// (simulate_rows_f64_wave); the others only get their keep flag. A large
// scan_min packs the in-band rows into few wavefronts, so that they take few
// issue slots from a float32 launch running beside them; scan_min = 1
// spreads them for the shortest latency. Workgroups that meet no in-band row
// never stage the observed series.
template <int NOISE, int DIST>
__device__ __forceinline__ void recheck_group(const RecheckArgs& r, const RowLds& l, int nr,
                                              bool& staged)
{
    const SimArgs& a = r.sim;
    if (!staged) {
        stage_obs_f64<DIST>(a.obs, a.T, l.lobs);
        staged = true;
    }
    __syncthreads();
    const double d64 = simulate_rows_f64_wave<NOISE, DIST>(
        nr, l.rth, l.rix, a.key, a.series, a.domain, a.P, a.A0, a.R0, a.D0, a.T, (double)a.scale,
        l.lobs, l.zs, l.xs, l.rw);
    const int lane = threadIdx.x;
    if (lane < nr) {
        const int64_t qq = l.rq[lane];
        r.keep[qq] = d64 <= (double)r.eps ? 1 : 0;
        r.dist[qq] = (float)d64;
        if (r.dist64) r.dist64[qq] = d64;
    }
    if (lane == 0 && r.rechecked) atomicAdd(r.rechecked, nr);
    __syncthreads();  // the row slots are refilled next
}

template <int NOISE, int DIST>
__global__ __launch_bounds__(64) void k_recheck_flags(RecheckArgs r)
{
    extern __shared__ double lds_r[];
    const int64_t count = *r.count;
    if (count > r.capacity) return;  // overflowed candidate set: left for the caller to rerun
    const RowLds l = row_lds(lds_r, r.sim.T, r.rows_max);
    int64_t per = (count + gridDim.x - 1) / gridDim.x;
    if (per < r.scan_min) per = r.scan_min;
    const int64_t q0 = (int64_t)blockIdx.x * per;
    if (q0 >= count) return;
    const int64_t q1 = q0 + per < count ? q0 + per : count;
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    bool staged = false;
    int nr = 0;  // rows gathered so far (wave-uniform)
    for (int64_t c0 = q0; c0 < q1; c0 += 64) {
        const int64_t q = c0 + lane;
        bool inb = false;
        if (q < q1) {
            const float d = r.dist[q];
            inb = r.all_rows || (d > r.band_lo && d <= r.band_hi);
            if (!inb) r.keep[q] = d <= r.eps ? 1 : 0;
        }
        uint64_t m = __ballot(inb);
        while (m) {
            // the lowest (rows_max - nr) in-band lanes join the group
            uint64_t take = 0;
            for (int room = r.rows_max - nr; room > 0 && m; --room) {
                const uint64_t b = m & (~m + 1ull);
                take |= b;
                m ^= b;
            }
            if ((take >> lane) & 1ull) {
                const int slot = nr + __popcll(take & below);
                l.rq[slot] = q;
                l.rix[slot] = (uint64_t)r.idx[q];
#pragma unroll
                for (int j = 0; j < 8; ++j) l.rth[8 * slot + j] = r.theta[8 * q + j];
            }
            nr += __popcll(take);
            if (nr == r.rows_max) {
                recheck_group<NOISE, DIST>(r, l, nr, staged);
                nr = 0;
            }
        }
    }
    if (nr > 0) recheck_group<NOISE, DIST>(r, l, nr, staged);
}

// Pass 2: stable in-place compaction of the kept rows, 256 rows at a time.
__global__ __launch_bounds__(256) void k_recheck_compact(RecheckArgs r)
{
    __shared__ int64_t base_sh;
    __shared__ int wave_tot[4];
    const int64_t count = *r.count;
    if (count > r.capacity) return;
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t c0 = 0; c0 < count; c0 += blockDim.x) {
        const int64_t q = c0 + threadIdx.x;
        const bool kp = q < count && r.keep[q];
        int64_t id = 0;
        float th[8], d = 0.0f, w = 0.0f;
        double d64 = 0.0;
        if (kp) {
            id = r.idx[q];
#pragma unroll
            for (int j = 0; j < 8; ++j) th[j] = r.theta[8 * q + j];
            d = r.dist[q];
            if (r.weight) w = r.weight[q];
            if (r.dist64) d64 = r.dist64[q];
        }
        const uint64_t m = __ballot(kp);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wave] = __popcll(m);
        __syncthreads();
        int off = 0, tot = 0;
        for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
            if (v < wave) off += wave_tot[v];
            tot += wave_tot[v];
        }
        const int64_t dst = base_sh + off + rank;
        __syncthreads();  // every row of this chunk is in registers before any write
        if (kp) {
            r.idx[dst] = id;
#pragma unroll
            for (int j = 0; j < 8; ++j) r.theta[8 * dst + j] = th[j];
            r.dist[dst] = d;
            if (r.weight) r.weight[dst] = w;
            if (r.dist64) r.dist64[dst] = d64;
        }
        __syncthreads();
        if (threadIdx.x == 0) base_sh += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *r.count = base_sh;
}

__global__ void k_zero_i32(int32_t* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}


// float64 distances of listed rows (sample idx[q], theta[q]), rows_per_wave
// consecutive rows at a time per wavefront, walked side by side in lanes.
struct RowsArgs {
    SimArgs sim;
    const int64_t* idx;
    double* dist64;
    int32_t rows_per_wave;
};

template <int NOISE, int DIST>
__global__ __launch_bounds__(64) void k_rows_f64(RowsArgs r)
{
    extern __shared__ double lds_w[];
    const SimArgs& a = r.sim;
    const int T = a.T, R = r.rows_per_wave;
    const RowLds l = row_lds(lds_w, T, R);
    stage_obs_f64<DIST>(a.obs, T, l.lobs);
    const int lane = threadIdx.x;
    for (int64_t q0 = (int64_t)blockIdx.x * R; q0 < a.n; q0 += (int64_t)gridDim.x * R) {
        const int nr = (int)(a.n - q0 < R ? a.n - q0 : R);
        if (lane < nr) {
            l.rix[lane] = (uint64_t)r.idx[q0 + lane];
#pragma unroll
            for (int j = 0; j < 8; ++j) l.rth[8 * lane + j] = a.theta[8 * (q0 + lane) + j];
        }
        __syncthreads();
        const double d64 = simulate_rows_f64_wave<NOISE, DIST>(
            nr, l.rth, l.rix, a.key, a.series, a.domain, a.P, a.A0, a.R0, a.D0, T,
            (double)a.scale, l.lobs, l.zs, l.xs, l.rw);
        if (lane < nr) r.dist64[q0 + lane] = d64;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// trajectory recording (float32 or float64 arithmetic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_state(int32_t* row, const State& s)
{
    row[0] = s.S; row[1] = s.I; row[2] = s.A; row[3] = s.R; row[4] = s.D; row[5] = s.Ru;
}

template <int NOISE, bool F64>
__global__ __launch_bounds__(SIM_BLOCK) void k_record(SimArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint64_t i = a.first + (uint64_t)k;
    float thv[8];
    load_or_draw_theta(a, false, k, i, thv);
    const Theta th = theta_from(thv);
    State s = init_state(th.ka, a.P, a.A0, a.R0, a.D0);
    int32_t* out = a.traj + (int64_t)6 * (a.T + 1) * k;
    store_state(out, s);
    const RatesF r = rates_f32(th);
    const float invP = 1.0f / (float)a.P;
    const float nc = noise_c(a.scale);
    for (int t = 1; t <= a.T; ++t) {
        const uint4 w = stream_words(a.key, i, a.series, ctr_word3((uint32_t)t, a.domain, 0));
        if (F64) {
            double z[5];
            normals_f64(w, z);
            day_step_f64<NOISE>(s, th, (double)a.P, (double)a.scale, z);
        } else {
            Noise32 z;
            normals_f32(w, nc, z);
            day_step_f32<NOISE>(s, r, invP, z);
        }
        store_state(out + 6 * t, s);
    }
}

// ---------------------------------------------------------------------------
// prior sampling
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SIM_BLOCK) void k_sample_prior(SimArgs a, float* theta)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    float th[8];
    prior_draw(a.key, a.first + (uint64_t)k, a.series, a.domain, a.lo, a.width, th);
    float4* p = reinterpret_cast<float4*>(theta + 8 * k);
    p[0] = make_float4(th[0], th[1], th[2], th[3]);
    p[1] = make_float4(th[4], th[5], th[6], th[7]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static abc_status fill_series(SimArgs& a, const abc_series* ser, const abc_model* m,
                              const abc_stream* st, uint64_t first, int64_t n)
{
    a.key = make_key(st->seed);
    a.domain = st->domain;
    a.series = st->series;
    a.first = first;
    a.n = n;
    a.P = (int32_t)ser->P;
    a.A0 = ser->A0;
    a.R0 = ser->R0;
    a.D0 = ser->D0;
    a.T = ser->T;
    a.obs = ser->obs;
    a.scale = m->noise_scale;
    return ABC_OK;
}

// float64 row kernels: one wavefront per workgroup, up to R rows side by side
// per wavefront, rows strided over the grid
constexpr int64_t ROW_WAVE_GRID = 2048;
static size_t row_wave_lds_bytes(int T, int R)
{
    return sizeof(double) * 3 * (size_t)T +
           (size_t)R * (sizeof(double) * 5 * ROW_WINDOW + sizeof(uint64_t) + sizeof(int64_t) +
                        sizeof(RowWalk) + sizeof(int32_t) * 3 * ROW_WINDOW + sizeof(float) * 8);
}
// Most rows per wavefront within an LDS budget (at least 1).
static int row_wave_rows_max(int T, size_t budget)
{
    int R = ROWS_PER_WAVE_MAX;
    while (R > 1 && row_wave_lds_bytes(T, R) > budget) --R;
    return R;
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + SIM_BLOCK - 1) / SIM_BLOCK); }

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Launch shape of the float32 refill kernel for the calling thread: samples
// per lane, workgroup size and resident workgroups per CU (0 = default).
struct LaunchConfig {
    int spl = 1;
    int block = 512;
    int blocks_per_cu = 2;
    int refill_min = 8;
};
static thread_local LaunchConfig g_launch;

// Resident-grid size for the refill kernel: enough workgroups to fill every
// CU several times over, never more than there are 64-sample chunks.
static unsigned refill_grid(int64_t n, int block, int blocks_per_cu)
{
    DeviceInfo info;
    const int num_cu = device_info(&info) == ABC_OK && info.num_cu > 0 ? info.num_cu : 256;
    const int64_t waves_needed = (n + 63) / 64;
    const int64_t per_block = block / 64;
    int64_t g = (int64_t)num_cu * blocks_per_cu;
    const int64_t need = (waves_needed + per_block - 1) / per_block;
    if (g > need) g = need;
    return (unsigned)(g > 0 ? g : 1);
}

// observed series | future-days bound table | ring (which first holds the
// float64 b_s and the segment sums staged for the table)
static size_t refill_lds_bytes(int T, int block, int lb_ntb)
{
    const size_t ring = sizeof(Slot) * 64 * (size_t)(block / 64);
    const size_t stage =
        lb_ntb > 0 ? sizeof(double) * (2 * (size_t)T + (size_t)LB_MAX_SEG * 2 * LB_Q) : 0;
    return sizeof(float) * (size_t)((3 * T + 3) & ~3) + sizeof(float) * 2 * LB_Q * (size_t)lb_ntb +
           (ring > stage ? ring : stage);
}

static size_t max_lds_per_block()
{
    DeviceInfo info;
    return device_info(&info) == ABC_OK && info.max_lds > 0 ? (size_t)info.max_lds : 65536;
}

template <int NOISE, int DIST, bool KAHAN, int SPL>
static void launch_f32_spl(const SimArgs& a, bool prior, hipStream_t s)
{
    const int block = g_launch.block;
    const size_t lds = refill_lds_bytes(a.T, block, a.lb_ntb);
    const dim3 g(refill_grid(a.n, block, g_launch.blocks_per_cu)), b(block);
    if (prior)
        hipLaunchKernelGGL((k_simulate_f32<NOISE, DIST, KAHAN, true, SPL>), g, b, lds, s, a);
    else
        hipLaunchKernelGGL((k_simulate_f32<NOISE, DIST, KAHAN, false, SPL>), g, b, lds, s, a);
}

template <int NOISE, int DIST, bool KAHAN>
static void launch_f32(const SimArgs& a, bool prior, hipStream_t s)
{
    // several samples per lane only for the paper's model and distance
    if constexpr (NOISE == 0 && DIST == 0) {
        switch (g_launch.spl) {
        case 2: launch_f32_spl<NOISE, DIST, KAHAN, 2>(a, prior, s); return;
        case 4: launch_f32_spl<NOISE, DIST, KAHAN, 4>(a, prior, s); return;
        case 8: launch_f32_spl<NOISE, DIST, KAHAN, 8>(a, prior, s); return;
        default: break;
        }
    }
    launch_f32_spl<NOISE, DIST, KAHAN, 1>(a, prior, s);
}

template <int NOISE, int DIST>
static void launch_f64(const SimArgs& a, bool prior, size_t lds, hipStream_t s)
{
    if (prior)
        hipLaunchKernelGGL((k_simulate_f64<NOISE, DIST, true>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
    else
        hipLaunchKernelGGL((k_simulate_f64<NOISE, DIST, false>), dim3(grid_for(a.n)),
                           dim3(SIM_BLOCK), lds, s, a);
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_sample_prior(const abc_prior* prior, const abc_stream* st,
                                       uint64_t first, int64_t n, float* theta, void* stream)
{
    SimArgs a{};
    abc_status rc = prior_lo_width(prior, a.lo, a.width);
    if (rc) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n = %lld < 0", (long long)n);
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(theta != nullptr && aligned16(theta), "theta must be a 16-byte aligned device pointer");
    a.key = make_key(st->seed);
    a.domain = st->domain;
    a.series = st->series;
    a.first = first;
    a.n = n;
    hipLaunchKernelGGL(k_sample_prior, dim3(grid_for(n)), dim3(SIM_BLOCK), 0, as_stream(stream),
                       a, theta);
    return check_launch("k_sample_prior");
}

extern "C" abc_status abc_simulate_distance(const abc_series* ser, const abc_model* model,
                                            const abc_stream* st, const float* theta,
                                            const abc_prior* prior, uint64_t first, int64_t n,
                                            float eps_exit, float* dist, double* dist64,
                                            unsigned long long* days, void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0 && n <= ((int64_t)1 << 36), "n = %lld outside [0, 2^36]", (long long)n);
    ABC_REQUIRE(!(eps_exit < 0.0f) && !isnan(eps_exit), "eps_exit must be >= 0 (or +INF)");
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(dist != nullptr, "dist is NULL");
    SimArgs a{};
    const bool use_prior = theta == nullptr;
    if (use_prior) {
        if ((rc = prior_lo_width(prior, a.lo, a.width))) return rc;
        for (int k = 0; k < 8; ++k)
            ABC_REQUIRE(prior->lo[k] >= 0.0f, "model rates must be non-negative: prior lo[%d] < 0", k);
    } else {
        ABC_REQUIRE(aligned16(theta), "theta must be 16-byte aligned");
        if (model->flags & ABC_SUPPORT) {
            if ((rc = prior_lo_width(prior, a.lo, a.width))) return rc;
            for (int k = 0; k < 8; ++k) a.hi[k] = prior->hi[k];
            a.box = 1;
        }
    }
    fill_series(a, ser, model, st, first, n);
    a.theta = theta;
    a.dist = dist;
    a.dist64 = dist64;
    a.days = days;
    a.refill_min = g_launch.refill_min;
    // Early-exit bounds with a relative margin that keeps every exited sample
    // strictly above eps_exit after the final square root and rounding.
    const double e2 = (double)eps_exit * (double)eps_exit;
    // the float32 log1p distance accumulates in log2 units: bound / ln(2)^2
    const double unit = (model->flags & ABC_DIST_RAW) ? 1.0 : 2.08136898100560809980;
    a.exit_f32 = isinf(eps_exit) ? INFINITY : (float)(e2 * unit * (1.0 + 0x1p-18));
    a.exit_f64 = isinf(eps_exit) ? (double)INFINITY : e2 * (1.0 + 1e-12);

    const hipStream_t s = as_stream(stream);
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const int distm = (model->flags & ABC_DIST_RAW) ? 1 : 0;
    if (model->flags & ABC_FP64) {
        const size_t lds = sizeof(double) * 3 * (size_t)a.T;
        if (noise == 0 && distm == 0) launch_f64<0, 0>(a, use_prior, lds, s);
        else if (noise == 0 && distm == 1) launch_f64<0, 1>(a, use_prior, lds, s);
        else if (noise == 1 && distm == 0) launch_f64<1, 0>(a, use_prior, lds, s);
        else launch_f64<1, 1>(a, use_prior, lds, s);
        return check_launch("k_simulate_f64");
    }
    // future-days bound for the log1p distance when there is an exit bound;
    // time blocks of 2^sh days keep the table within LB_MAX_BLOCKS rows
    if (distm == 0 && !isinf(eps_exit) && !(model->flags & ABC_NO_BOUND)) {
        int sh = 0;
        while ((a.T >> sh) + 1 > LB_MAX_BLOCKS) ++sh;
        a.lb_sh = sh;
        a.lb_ntb = (a.T >> sh) + 1;
        if (refill_lds_bytes(a.T, g_launch.block, a.lb_ntb) > max_lds_per_block()) a.lb_ntb = 0;
    }
    const size_t lds = refill_lds_bytes(a.T, g_launch.block, a.lb_ntb);
    if (lds > max_lds_per_block())
        return set_error(ABC_EUNSUPPORTED, "T = %d with workgroup size %d needs %zu B of LDS (> %zu)",
                         a.T, g_launch.block, lds, max_lds_per_block());
    const bool kahan = (model->flags & ABC_KAHAN) != 0;
    if (kahan) {
        if (noise == 0 && distm == 0) launch_f32<0, 0, true>(a, use_prior, s);
        else if (noise == 0 && distm == 1) launch_f32<0, 1, true>(a, use_prior, s);
        else if (noise == 1 && distm == 0) launch_f32<1, 0, true>(a, use_prior, s);
        else launch_f32<1, 1, true>(a, use_prior, s);
    } else {
        if (noise == 0 && distm == 0) launch_f32<0, 0, false>(a, use_prior, s);
        else if (noise == 0 && distm == 1) launch_f32<0, 1, false>(a, use_prior, s);
        else if (noise == 1 && distm == 0) launch_f32<1, 0, false>(a, use_prior, s);
        else launch_f32<1, 1, false>(a, use_prior, s);
    }
    return check_launch("k_simulate_f32");
}

extern "C" abc_status abc_simulate_record(const abc_series* ser, const abc_model* model,
                                          const abc_stream* st, const float* theta,
                                          uint64_t first, int64_t n, int32_t* traj, void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, false))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n = %lld < 0", (long long)n);
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(theta != nullptr && aligned16(theta), "theta must be a 16-byte aligned device pointer");
    ABC_REQUIRE(traj != nullptr, "traj is NULL");
    SimArgs a{};
    fill_series(a, ser, model, st, first, n);
    a.theta = theta;
    a.traj = traj;
    const hipStream_t s = as_stream(stream);
    const bool f64 = (model->flags & ABC_FP64) != 0;
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const dim3 g(grid_for(n)), b(SIM_BLOCK);
    if (f64) {
        if (noise) hipLaunchKernelGGL((k_record<1, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_record<0, true>), g, b, 0, s, a);
    } else {
        if (noise) hipLaunchKernelGGL((k_record<1, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_record<0, false>), g, b, 0, s, a);
    }
    return check_launch("k_record");
}

extern "C" abc_status abc_set_launch_config(int32_t spl, int32_t block, int32_t blocks_per_cu)
{
    if (spl == 0) spl = 1;
    if (block == 0) block = 512 / spl < 64 ? 64 : 512 / spl;
    if (blocks_per_cu == 0) blocks_per_cu = 2;
    ABC_REQUIRE(spl == 1 || spl == 2 || spl == 4 || spl == 8, "spl must be 1, 2, 4 or 8");
    ABC_REQUIRE(block >= 64 && block <= 1024 / spl && block % 64 == 0,
                "block must be a multiple of 64 in [64, 1024/spl]");
    ABC_REQUIRE(blocks_per_cu >= 1 && blocks_per_cu <= 64, "blocks_per_cu must be in [1, 64]");
    g_launch.spl = spl;
    g_launch.block = block;
    g_launch.blocks_per_cu = blocks_per_cu;
    return ABC_OK;
}

extern "C" abc_status abc_get_launch_config(int32_t* spl, int32_t* block, int32_t* blocks_per_cu)
{
    ABC_REQUIRE(spl && block && blocks_per_cu, "NULL output pointer");
    *spl = g_launch.spl;
    *block = g_launch.block;
    *blocks_per_cu = g_launch.blocks_per_cu;
    return ABC_OK;
}

namespace abc {
abc_status recheck_band(const abc_series* ser, const abc_model* model, const abc_stream* st,
                        float eps, float band_w, int64_t capacity, int64_t* idx, float* theta,
                        float* dist, float* weight, int64_t* count, int32_t* rechecked,
                        void* stream, size_t lds_budget, int64_t grid_max, int32_t scan_min,
                        double* dist64, bool all_rows)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(!isnan(eps) && eps >= 0.0f, "eps must be >= 0 (or +INF)");
    ABC_REQUIRE(isfinite(band_w) && band_w >= 0.0f && band_w < 1.0f, "band_w must be in [0, 1)");
    ABC_REQUIRE(capacity >= 0, "capacity < 0");
    ABC_REQUIRE(count != nullptr, "count is NULL");
    if (capacity == 0) return ABC_OK;
    ABC_REQUIRE(idx && theta && dist, "idx/theta/dist NULL");
    const int rows_max = row_wave_rows_max(ser->T, lds_budget);
    const size_t lds = row_wave_lds_bytes(ser->T, rows_max);
    ABC_REQUIRE(lds <= max_lds_per_block(), "T too long for the float64 recheck");
    const hipStream_t s = as_stream(stream);
    RecheckArgs r{};
    fill_series(r.sim, ser, model, st, 0, 0);
    r.eps = eps;
    r.band_lo = (float)((double)eps * (1.0 - (double)band_w));
    r.band_hi = (float)((double)eps * (1.0 + (double)band_w));
    r.capacity = capacity;
    r.idx = idx;
    r.theta = theta;
    r.dist = dist;
    r.weight = weight;
    r.count = count;
    r.rechecked = rechecked;
    r.rows_max = rows_max;
    r.scan_min = scan_min < 1 ? 1 : scan_min;
    r.all_rows = all_rows ? 1 : 0;
    r.dist64 = dist64;
    void* scratch = nullptr;
    if ((rc = stream_scratch(s, (size_t)capacity, &scratch))) return rc;
    r.keep = reinterpret_cast<uint8_t*>(scratch);
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const int distm = (model->flags & ABC_DIST_RAW) ? 1 : 0;
    if (rechecked) hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, rechecked);
    const dim3 g((unsigned)(capacity < grid_max ? capacity : grid_max)), b(64);
    if (noise == 0 && distm == 0) hipLaunchKernelGGL((k_recheck_flags<0, 0>), g, b, lds, s, r);
    else if (noise == 0) hipLaunchKernelGGL((k_recheck_flags<0, 1>), g, b, lds, s, r);
    else if (distm == 0) hipLaunchKernelGGL((k_recheck_flags<1, 0>), g, b, lds, s, r);
    else hipLaunchKernelGGL((k_recheck_flags<1, 1>), g, b, lds, s, r);
    rc = check_launch("k_recheck_flags");
    if (rc == ABC_OK) {
        hipLaunchKernelGGL(k_recheck_compact, dim3(1), dim3(256), 0, s, r);
    }
    if (rc == ABC_OK) rc = check_launch("k_recheck_compact");
    return rc;
}
}  // namespace abc

extern "C" abc_status abc_recheck_band(const abc_series* ser, const abc_model* model,
                                       const abc_stream* st, float eps, float band_w,
                                       int64_t capacity, int64_t* idx, float* theta, float* dist,
                                       float* weight, int64_t* count, int32_t* rechecked,
                                       void* stream)
{
    return recheck_band(ser, model, st, eps, band_w, capacity, idx, theta, dist, weight, count,
                        rechecked, stream, ROW_LDS_BESIDE, ROW_WAVE_GRID, ROW_SCAN_BESIDE,
                        nullptr, false);
}

extern "C" abc_status abc_simulate_rows_f64(const abc_series* ser, const abc_model* model,
                                            const abc_stream* st, const int64_t* idx,
                                            const float* theta, int64_t n, double* dist64,
                                            void* stream)
{
    abc_status rc;
    if ((rc = check_series(ser, true))) return rc;
    if ((rc = check_model(model))) return rc;
    if ((rc = check_stream_sel(st))) return rc;
    ABC_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return ABC_OK;
    ABC_REQUIRE(idx && theta && dist64, "idx/theta/dist64 NULL");
    const int64_t want = (n + ROW_WAVE_TARGET - 1) / ROW_WAVE_TARGET;
    const int rmax = row_wave_rows_max(ser->T, ROW_LDS_ALONE);
    const int rows = (int)(want < rmax ? want : rmax);
    const size_t lds = row_wave_lds_bytes(ser->T, rows);
    ABC_REQUIRE(lds <= max_lds_per_block(), "T too long for the float64 path");
    RowsArgs r{};
    fill_series(r.sim, ser, model, st, 0, n);
    r.sim.theta = theta;
    r.idx = idx;
    r.dist64 = dist64;
    r.rows_per_wave = rows;
    const hipStream_t s = as_stream(stream);
    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const int distm = (model->flags & ABC_DIST_RAW) ? 1 : 0;
    const int64_t waves = (n + rows - 1) / rows;
    const dim3 g((unsigned)(waves < ROW_WAVE_GRID ? waves : ROW_WAVE_GRID)), b(64);
    if (noise == 0 && distm == 0) hipLaunchKernelGGL((k_rows_f64<0, 0>), g, b, lds, s, r);
    else if (noise == 0) hipLaunchKernelGGL((k_rows_f64<0, 1>), g, b, lds, s, r);
    else if (distm == 0) hipLaunchKernelGGL((k_rows_f64<1, 0>), g, b, lds, s, r);
    else hipLaunchKernelGGL((k_rows_f64<1, 1>), g, b, lds, s, r);
    return check_launch("k_rows_f64");
}

extern "C" abc_status abc_set_refill_min(int32_t lanes)
{
    if (lanes == 0) lanes = 8;
    ABC_REQUIRE(lanes >= 1 && lanes <= 64, "lanes must be in [1, 64]");
    g_launch.refill_min = lanes;
    return ABC_OK;
}

extern "C" int32_t abc_get_refill_min(void) { return g_launch.refill_min; }
