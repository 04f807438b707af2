// Several series in one persistent float32 simulate+distance launch, and its
// C-ABI entry point abc_simulate_distance_multi.
//
// The per-series launches of abc_simulate_distance each end with a tail in
// which the last trajectories of every wavefront's queue run to their last
// day while most lanes of the device are idle. Here the 64-sample chunks of
// all series form one queue: each wavefront owns a fixed stride of chunks
// over it, takes a chunk's 64 samples into its ring (prior draw, rates,
// initial state and the per-sample Philox words, prepared by the whole
// wavefront), and every lane carries the series of the sample it holds --
// its horizon, observed rows and future-days bound table in LDS, tolerance
// and Philox series word. Series are laid out in the queue longest horizon
// first, so a launch ends on its shortest trajectories and pays one tail.
// The day step, the early exit and the distance are those of the one-series
// kernel: every distance is bit-identical to abc_simulate_distance's.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "bound.hpp"
#include "common.hpp"
#include "model.hpp"

namespace abc {

constexpr int MS_MAX = ABC_MULTI_MAX;

struct MSeries {
    int32_t P, A0, R0, D0, T;
    uint32_t series;   // Philox series word
    uint32_t u0, b1;   // its per-series Philox constants
    float invP;
    float exit_f32;    // squared-distance early-exit bound in log2 units (or raw)
    int32_t obs_off;   // float offset of the observed rows [3][T] in LDS
    int32_t tab_off;   // float offset of the bound table [2][ntb][LB_Q] in LDS, -1: none
    int32_t ntb, lb_sh;
    int64_t chunk0;    // first chunk of the series in the launch's queue
    int64_t n;
    uint64_t first;
    const int32_t* obs;
    float* dist;
};

struct MultiArgs {
    MSeries s[MS_MAX];
    int32_t m;
    int32_t refill_min;
    int64_t nchunks;
    float lo[8];
    float width[8];
    Key key;
    uint32_t domain;
    float scale;
    int32_t obs_words;  // floats of all observed rows (a multiple of 4)
    int32_t tab_words;  // floats of all bound tables (a multiple of 4)
    unsigned long long* days;
};

// What a lane reads from LDS when it starts a sample of series j.
struct alignas(16) SerLds {
    float invP, exitb;
    int32_t T, obs_off, tab_r, tab_d, lb_sh;
    uint32_t b1;
    float* dist;
    int32_t A0, R0, D0, room;  // room = P - A0 - R0 - D0 (S0 + I0)
};

// One prepared sample: rates, I0 and the per-sample Philox words. Its series
// and offset follow from the chunk in the ring, which is wave-uniform, so they
// are not stored (48 bytes a slot).
struct alignas(16) MSlot {
    float a0, al, n, be, ga, de, bh;
    int32_t i0;
    uint32_t c1base, g3, h3, f3;
};

struct MLane {
    State s;
    RatesF r;
    PhiloxDays ph;
    int64_t k;
    int32_t t;  // the day the lane simulates next; 0: no sample (idle)
    float acc, comp;
    int32_t ls;
    // the lane's series, cached at the start of each sample (tr, td: its
    // bound tables for R and D, tr null without one)
    int32_t T, obs_off, lb_sh;
    const float* tr;
    const float* td;
    float invP, exitb;
    uint32_t b1;
};

template <int NOISE, int DIST, bool KAHAN>
__global__ __launch_bounds__(1024) void k_simulate_multi_f32(MultiArgs a)
{
    constexpr int RING = 64;
    extern __shared__ float lds_f[];
    float* tabs = lds_f + a.obs_words;
    SerLds* ser = reinterpret_cast<SerLds*>(tabs + a.tab_words);
    MSlot* ring_all = reinterpret_cast<MSlot*>(ser + MS_MAX);

    // observed rows of every series: log2(1 + O) (or O for the raw distance)
    for (int j = 0; j < a.m; ++j) {
        const MSeries& sj = a.s[j];
        for (int q = threadIdx.x; q < 3 * sj.T; q += blockDim.x) {
            const int32_t O = sj.obs[q];
            if (DIST == 0)
                lds_f[sj.obs_off + q] = (float)(log1p((double)O) * 1.44269504088896340736);
            else
                lds_f[sj.obs_off + q] = __int_as_float(O);
        }
    }
    if (threadIdx.x < (unsigned)a.m) {
        const MSeries& sj = a.s[threadIdx.x];
        SerLds e;
        e.invP = sj.invP;
        e.exitb = sj.exit_f32;
        e.T = sj.T;
        e.obs_off = sj.obs_off;
        e.tab_r = sj.tab_off;
        e.tab_d = sj.tab_off + sj.ntb * LB_Q;
        e.lb_sh = sj.lb_sh;
        e.b1 = sj.b1;
        e.dist = sj.dist;
        e.A0 = sj.A0;
        e.R0 = sj.R0;
        e.D0 = sj.D0;
        e.room = sj.P - (sj.A0 + sj.R0 + sj.D0);
        ser[threadIdx.x] = e;
    }
    if (DIST == 0) {
        // future-days bound tables, one series at a time; b_s of R and D in
        // float64 staged where the ring will live
        double* stage = reinterpret_cast<double*>(ring_all);
        for (int j = 0; j < a.m; ++j) {
            const MSeries& sj = a.s[j];
            if (sj.tab_off < 0) continue;
            __syncthreads();
            for (int q = threadIdx.x; q < 2 * sj.T; q += blockDim.x)
                stage[q] = log1p((double)sj.obs[sj.T + q]) * 1.44269504088896340736;
            __syncthreads();
            build_future_bound(stage, sj.T, sj.lb_sh, sj.ntb, (double)sj.exit_f32, tabs + sj.tab_off);
        }
    }
    __syncthreads();

    __builtin_amdgcn_s_setprio(1);
    const int lane = threadIdx.x & 63;
    // the wavefront index is uniform over the wave: kept scalar, so is
    // everything of the queue derived from it
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    MSlot* ring = ring_all + wv * RING;
    const int64_t wg = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    if (wg >= a.nchunks) return;
    // queue positions of this wave (the host keeps them within 32 bits); its
    // j-th chunk is wg + j nw
    const uint32_t Q = (uint32_t)(((a.nchunks - 1 - wg) / nw + 1) << 6);
    const float nc = noise_c(a.scale);
    const float dscale = DIST == 0 ? 0.693147180559945309417f : 1.0f;
    const uint32_t wdom = a.domain << 4;

    // the chunk in the ring (wave-uniform): its series, the offset of its
    // first sample in that series, and how many of its 64 positions hold a
    // sample (fewer only in a series' last chunk)
    int cur_ls = 0;
    int64_t cur_base = 0;
    uint32_t cur_valid = 0;
    // chunk c into the ring: series by the chunk ranges
    auto fill = [&](int64_t c) {
        int ls = 0;
        for (int j = 1; j < a.m; ++j)
            if (c >= a.s[j].chunk0) ls = j;
        ls = __builtin_amdgcn_readfirstlane(ls);
        const MSeries& sj = a.s[ls];
        cur_ls = ls;
        cur_base = (c - sj.chunk0) << 6;
        cur_valid = (uint32_t)min(sj.n - cur_base, (int64_t)64);
        const int64_t k = cur_base + lane;
        MSlot& sl = ring[lane];
        if (k < sj.n) {
            const uint64_t i = sj.first + (uint64_t)k;
            float thv[8];
            prior_draw(a.key, i, sj.series, a.domain, a.lo, a.width, thv);
            const Theta th = theta_from(thv);
            const RatesF r = rates_f32(th);
            const State s0 = init_state(th.ka, sj.P, sj.A0, sj.R0, sj.D0);
            PhiloxDays ph;
            ph.begin(i, sj.u0, a.key);
            sl.a0 = r.a0; sl.al = r.al; sl.n = r.n; sl.be = r.be;
            sl.ga = r.ga; sl.de = r.de; sl.bh = r.bh; sl.i0 = s0.I;
            sl.c1base = ph.c1base; sl.g3 = ph.g3; sl.h3 = ph.h3; sl.f3 = ph.f3;
        }
    };

    uint32_t qb = 0;
    uint32_t filled = 0xFFFFFFFFu;
    MLane l;
    l.t = 0;
    uint32_t days_done = 0;

    while (true) {
        // refill: the idle lanes take the next queue positions in lane order,
        // once at least refill_min of them are idle; a pass may span the end
        // of one chunk and the start of the next
        bool want = l.t == 0;
        uint64_t m = __ballot(want);
        if (__popcll(m) >= a.refill_min) {
            while (m != 0ull && qb < Q) {
                const uint32_t jc = qb >> 6;
                if (jc != filled) {
                    fill(wg + (int64_t)jc * nw);
                    filled = jc;
                }
                const uint32_t off = qb & 63u;
                const uint32_t avail = 64u - off;
                // lanes of m below this one
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const bool take = want && rank < avail;
                const uint32_t pos = off + rank;
                if (take && pos < cur_valid) {
                    const MSlot sl = ring[pos];
                    const SerLds e = ser[cur_ls];
                    l.r = RatesF{sl.a0, sl.al, sl.n, sl.be, sl.ga, sl.de, sl.bh};
                    l.s.A = e.A0; l.s.R = e.R0; l.s.D = e.D0; l.s.Ru = 0;
                    l.s.I = sl.i0;
                    l.s.S = e.room - sl.i0;
                    l.ph.c1base = sl.c1base; l.ph.g3 = sl.g3; l.ph.h3 = sl.h3; l.ph.f3 = sl.f3;
                    l.k = cur_base + (int64_t)pos;
                    l.ls = cur_ls;
                    l.T = e.T; l.obs_off = e.obs_off;
                    l.tr = e.tab_r >= 0 ? tabs + e.tab_r : nullptr;
                    l.td = tabs + e.tab_d;
                    l.lb_sh = e.lb_sh; l.invP = e.invP; l.exitb = e.exitb; l.b1 = e.b1;
                    l.t = 1;
                    l.acc = 0.0f;
                    l.comp = 0.0f;
                }
                want = want && !take;
                const uint32_t cnt = (uint32_t)__popcll(m);
                qb += cnt < avail ? cnt : avail;
                m = __ballot(want);
            }
        }
        if (__ballot(l.t != 0) == 0ull && qb >= Q) break;
        if (l.t != 0) {
            const int t = l.t;
            const uint4 w = l.ph.day(((uint32_t)t << 8) | wdom, l.b1, a.key);
            Noise32 z;
            normals_f32(w, nc, z);
            day_step_f32<NOISE>(l.s, l.r, l.invP, z);
            const int32_t X[3] = {l.s.A, l.s.R, l.s.D};
            float lx[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int q = l.obs_off + c * l.T + t - 1;
                float d;
                if (DIST == 0) {
                    lx[c] = log2p1_count_f32(X[c]);
                    d = lx[c] - lds_f[q];
                } else {
                    d = (float)(X[c] - __float_as_int(lds_f[q]));
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
            if (DIST == 0 && l.tr != nullptr) {
                const int row = (t >> l.lb_sh) * LB_Q;
                const int qr = (int)fmaf(lx[1], 2.0f, -0x1p-12f);
                const int qd = (int)fmaf(lx[2], 2.0f, -0x1p-12f);
                lb = l.tr[row + qr] + l.td[row + qd];
            }
            const bool exited = l.acc + lb > l.exitb;
            if (exited || t == l.T) {
                const float dd = exited ? INFINITY : finish_distance_f32(l.acc, dscale);
                ser[l.ls].dist[l.k] = dd;
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

static size_t multi_lds_bytes(int obs_words, int tab_words, int block, int stage_doubles)
{
    const size_t ring = sizeof(MSlot) * 64 * (size_t)(block / 64);
    const size_t stage = sizeof(double) * (size_t)stage_doubles;
    return sizeof(float) * ((size_t)obs_words + (size_t)tab_words) + sizeof(SerLds) * MS_MAX +
           (ring > stage ? ring : stage);
}

template <int NOISE, int DIST, bool KAHAN>
static void launch_multi(const MultiArgs& a, unsigned grid, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_simulate_multi_f32<NOISE, DIST, KAHAN>), dim3(grid), dim3(block), lds, s, a);
}

}  // namespace abc

using namespace abc;

extern "C" abc_status abc_simulate_distance_multi(const abc_sim_job* jobs, int32_t m,
                                                  const abc_model* model, const abc_prior* prior,
                                                  uint64_t seed, uint32_t domain,
                                                  unsigned long long* days, void* stream)
{
    abc_status rc;
    ABC_REQUIRE(jobs != nullptr && m >= 1 && m <= MS_MAX, "need 1 <= m <= %d jobs", MS_MAX);
    if ((rc = check_model(model))) return rc;
    ABC_REQUIRE((model->flags & (ABC_FP64 | ABC_SUPPORT)) == 0,
                "the multi-series launch runs the float32 path with in-kernel prior draws "
                "(ABC_FP64 and ABC_SUPPORT are not options here)");
    ABC_REQUIRE(domain <= 15u, "domain %u > 15", domain);
    MultiArgs a{};
    if ((rc = prior_lo_width(prior, a.lo, a.width))) return rc;
    for (int k = 0; k < 8; ++k)
        ABC_REQUIRE(prior->lo[k] >= 0.0f, "model rates must be non-negative: prior lo[%d] < 0", k);
    int64_t total = 0;
    for (int j = 0; j < m; ++j) {
        const abc_sim_job& jb = jobs[j];
        if ((rc = check_series(jb.ser, true))) return set_error(rc, "job %d: %s", j, abc_last_error());
        ABC_REQUIRE(jb.n >= 0 && jb.n <= ((int64_t)1 << 36), "job %d: n = %lld outside [0, 2^36]",
                    j, (long long)jb.n);
        ABC_REQUIRE(!(jb.eps_exit < 0.0f) && !isnan(jb.eps_exit), "job %d: eps_exit must be >= 0 (or +INF)", j);
        ABC_REQUIRE(jb.n == 0 || jb.dist != nullptr, "job %d: dist is NULL", j);
        total += jb.n;
    }
    ABC_REQUIRE(total <= ((int64_t)1 << 36), "%lld samples in total exceed 2^36", (long long)total);
    if (total == 0) return ABC_OK;

    const int noise = (model->flags & ABC_NOISE_LITERAL) ? 1 : 0;
    const int distm = (model->flags & ABC_DIST_RAW) ? 1 : 0;
    const bool kahan = (model->flags & ABC_KAHAN) != 0;
    const bool bound = distm == 0 && !(model->flags & ABC_NO_BOUND);

    // queue order: longest horizon first (stable), jobs with samples only
    std::vector<int> order;
    for (int j = 0; j < m; ++j)
        if (jobs[j].n > 0) order.push_back(j);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return jobs[x].ser->T > jobs[y].ser->T; });
    a.m = (int32_t)order.size();
    a.key = make_key(seed);
    a.domain = domain;
    a.scale = model->noise_scale;
    a.days = days;
    int32_t spl = 1, block = 512, bpc = 2;
    abc_get_launch_config(&spl, &block, &bpc);
    a.refill_min = abc_get_refill_min();
    int obs_words = 0, maxT = 0;
    int64_t chunk = 0;
    std::vector<int> sh(a.m, 0), ntb(a.m, 0);
    for (int q = 0; q < a.m; ++q) {
        const abc_sim_job& jb = jobs[order[q]];
        MSeries& s = a.s[q];
        s.P = (int32_t)jb.ser->P;
        s.A0 = jb.ser->A0;
        s.R0 = jb.ser->R0;
        s.D0 = jb.ser->D0;
        s.T = jb.ser->T;
        s.series = jb.series;
        const uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)jb.series;
        s.u0 = (uint32_t)(p1 >> 32) ^ a.key.k0;
        s.b1 = (uint32_t)p1 ^ (a.key.k0 + PH_W0);
        s.invP = 1.0f / (float)jb.ser->P;
        // the same exit bound as abc_simulate_distance, in log2 units for log1p
        const double e2 = (double)jb.eps_exit * (double)jb.eps_exit;
        const double unit = distm ? 1.0 : 2.08136898100560809980;
        s.exit_f32 = isinf(jb.eps_exit) ? INFINITY : (float)(e2 * unit * (1.0 + 0x1p-18));
        s.obs_off = obs_words;
        obs_words += 3 * s.T;
        s.chunk0 = chunk;
        chunk += (jb.n + 63) >> 6;
        s.n = jb.n;
        s.first = jb.first;
        s.obs = jb.ser->obs;
        s.dist = jb.dist;
        if (s.T > maxT) maxT = s.T;
        if (bound && !isinf(jb.eps_exit)) {
            while ((s.T >> sh[q]) + 1 > LB_MAX_BLOCKS) ++sh[q];
            ntb[q] = (s.T >> sh[q]) + 1;
        }
    }
    a.nchunks = chunk;
    a.obs_words = (obs_words + 3) & ~3;
    const int stage_doubles = 2 * maxT + LB_MAX_SEG * 2 * LB_Q;
    DeviceInfo info;
    if ((rc = device_info(&info))) return rc;
    const int num_cu = info.num_cu, max_lds = info.max_lds;
    // bound tables: coarser time blocks for the series with the most rows until
    // blocks_per_cu workgroups fit a CU's LDS (160 KiB) and one fits the
    // workgroup limit; without room at all, no tables
    auto tab_words = [&]() {
        int w = 0;
        for (int q = 0; q < a.m; ++q) w += 2 * LB_Q * ntb[q];
        return w;
    };
    const size_t lds_target = std::min((size_t)max_lds, (size_t)(163840 / (bpc > 0 ? bpc : 1)));
    while (multi_lds_bytes(a.obs_words, tab_words(), block, stage_doubles) > lds_target) {
        int qmax = -1;
        for (int q = 0; q < a.m; ++q)
            if (ntb[q] > 1 && (qmax < 0 || ntb[q] > ntb[qmax])) qmax = q;
        if (qmax < 0) break;
        ++sh[qmax];
        ntb[qmax] = (a.s[qmax].T >> sh[qmax]) + 1;
    }
    if (multi_lds_bytes(a.obs_words, tab_words(), block, stage_doubles) > (size_t)max_lds)
        for (int q = 0; q < a.m; ++q) ntb[q] = 0;
    int tw = 0;
    for (int q = 0; q < a.m; ++q) {
        a.s[q].ntb = ntb[q];
        a.s[q].lb_sh = sh[q];
        a.s[q].tab_off = ntb[q] > 0 ? tw : -1;
        tw += 2 * LB_Q * ntb[q];
    }
    a.tab_words = tw;
    const size_t lds = multi_lds_bytes(a.obs_words, a.tab_words, block, stage_doubles);
    if (lds > (size_t)max_lds)
        return set_error(ABC_EUNSUPPORTED, "%d series with %d observed days need %zu B of LDS "
                         "per workgroup of %d (> %d)", a.m, obs_words, lds, block, max_lds);
    // resident workgroups: what the LDS allows per CU, at most blocks_per_cu
    int per_cu = (int)(163840 / lds);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > bpc) per_cu = bpc;
    const int64_t need = (a.nchunks + block / 64 - 1) / (block / 64);
    int64_t g = (int64_t)num_cu * per_cu;
    if (g > need) g = need;
    const hipStream_t s = as_stream(stream);
    const unsigned grid = (unsigned)g;
    if (kahan) {
        if (noise == 0 && distm == 0) launch_multi<0, 0, true>(a, grid, block, lds, s);
        else if (noise == 0) launch_multi<0, 1, true>(a, grid, block, lds, s);
        else if (distm == 0) launch_multi<1, 0, true>(a, grid, block, lds, s);
        else launch_multi<1, 1, true>(a, grid, block, lds, s);
    } else {
        if (noise == 0 && distm == 0) launch_multi<0, 0, false>(a, grid, block, lds, s);
        else if (noise == 0) launch_multi<0, 1, false>(a, grid, block, lds, s);
        else if (distm == 0) launch_multi<1, 0, false>(a, grid, block, lds, s);
        else launch_multi<1, 1, false>(a, grid, block, lds, s);
    }
    return check_launch("k_simulate_multi_f32");
}
