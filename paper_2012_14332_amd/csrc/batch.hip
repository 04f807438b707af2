// Batched persistent rejection ABC over many observed series of uneven
// length and population (Sec. 3.1 "iterate until the required number of
// accepted samples"), run as overlapping rounds on two streams, and its C-ABI entry
// point abc_batch_run.
//
// Round structure (all decisions on the device):
//   k_batch_plan   one workgroup: series whose float32 accepts
//                  (d <= eps (1 - 1e-5)) are below their target (first
//                  Q + margin) share the round's samples evenly, each
//                  capped by what its target still needs; each gets the
//                  next contiguous index range of its own stream. Plan p
//                  sees the counts of rounds up to p - 2 only, so round p - 1 can
//                  still run while it plans, and round p starts on the
//                  workgroup slots round p - 1 frees at its end: the rounds
//                  alternate between two streams and overlap their tails.
//   k_batch_round  persistent grid: every wavefront walks a fixed share of
//                  the round's 64-sample chunks with lane refill. Lanes carry
//                  their own series (T, P, tolerance, stream words), and the
//                  observed series of the whole batch sit in LDS, so a lane
//                  never waits for the rest of its wave to change series.
//                  A finished sample with d <= eps (1 + w) is appended to its
//                  series' candidate list; d <= eps (1 - 1e-5) also counts
//                  as a float32 accept toward the series' target.
// Because each series consumes its indices as a prefix, the first Q
// accepted samples by index are exact once Q accepts exist among the
// candidates: the finalisation decides the band candidates in float64, sorts
// by index and keeps the first Q; a series left short continues its stream
// with a higher target and is finalised again. The outcome does not depend
// on the launch shape.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "model.hpp"
#include "proposal.hpp"

namespace abc {

constexpr int BT_MAX_SERIES = 256;
constexpr int BT_RING = 64;  // ring slots per wave (one chunk)

struct SeriesDesc {         // device, per series, constant over the run
    int32_t T, P, A0, R0, D0;
    int32_t obs_off;        // offset of [3][T] log2(1 + O) floats in the obs table
    int32_t room;           // P - A0 - R0 - D0
    uint32_t series_id;     // stream series (counter word 2)
    float invP;
    float exit2;            // early-exit bound on the log2-unit sum
    float eps_hi, eps_lo, eps;
    uint32_t u0, b1;        // wave-uniform Philox words of this series
    float eps_cnt;          // float32 accepts with d <= eps_cnt count toward the target
};

constexpr int BT_SLOTS = 3;  // round p counts into slot p % 3 until plan p + 2 folds it
constexpr int BT_MAX_PHASES = 8;  // finalisations of one run (see abc_batch_run)
// Float32 accepts within this relative distance below eps do not count
// toward a series' target. Float32 and float64 distances differ by a few
// 1e-6 relative near eps, and identical trajectories (an atom of the distance
// distribution) share one distance: when eps is an atom's float32 distance,
// float64 puts all of the atom on one side of eps, often the far one.
constexpr double BT_TIE = 1e-5;
thread_local int32_t g_batch_margin = 0;  // abc_set_batch_margin; 0: the default

struct SeriesState {        // device, per series
    int64_t next;           // next sample index of the stream (assigned to some round)
    int64_t done;           // samples of the folded rounds
    int32_t acc;            // samples with float32 d <= eps_cnt so far (every finished sample)
    int32_t cand;           // candidate rows handed out so far (may exceed capacity)
    int32_t acc_f;          // float32 accepts of the folded rounds
    int32_t cand_f;         // candidates of the folded rounds
    int32_t target;         // the series takes samples until acc reaches this
    int32_t pad;
    int32_t rc_acc[BT_SLOTS];      // per-round counts, by slot
    int32_t rc_cand[BT_SLOTS];
    int64_t n_slot[BT_SLOTS];      // samples assigned to the round of each slot
};

struct RoundTable {
    int32_t n_active;
    int32_t total_chunks;
    int32_t done;
    int32_t pad;
    int32_t s[BT_MAX_SERIES];
    int32_t n[BT_MAX_SERIES];
    int32_t chunk0[BT_MAX_SERIES + 1];
    int64_t first[BT_MAX_SERIES];
};

struct BatchArgs {
    int32_t m;
    int32_t quota;
    int32_t target0;        // first target of every series' float32 accepts (quota + margin)
    int64_t round_size;
    int64_t max_samples;    // per series
    int32_t cand_cap;       // candidate rows per series
    int32_t obs_words;      // floats in the obs table
    Key key;
    uint32_t domain;
    float lo[8], width[8];
    const SeriesDesc* desc;
    SeriesState* state;
    RoundTable* table;      // this round's table (two, alternating with the round's parity)
    int32_t round;          // round index p (its count slot is p % BT_SLOTS)
    const float* obs_table; // [obs_words]
    int64_t* cand_idx;      // [m][cand_cap]
    float* cand_dist;       // [m][cand_cap]
    int32_t* flag_dev;      // 1 once no series needs more samples
    unsigned long long* days;
    float nc;               // -2 ln(2) s^2 of the Box-Muller radius
    float scale;
    int32_t refill_min;     // refill a wave's idle lanes once at least this many are idle
    const int32_t* order;   // [m] series in planning order (longest horizon first)
    const float* mix;       // null: prior draws; else [m][136] proposal rows (learned proposal)
    const MixTable* tables; // [m] truncated-mixture tables of the rows
    ProposalBox prop;
    uint32_t prop_domain;   // stream domain of the proposal draws
};

// theta of sample i of series s (desc d): the prior draw, or the learned
// proposal's draw with its importance weight
// (MIX: the learned proposal is in use; a compile-time switch so that the
// prior-only round kernel does not carry the proposal's code and registers)
template <bool MIX = true>
__device__ __forceinline__ float batch_theta(const BatchArgs& a, int s, const SeriesDesc& d, uint64_t i,
                                             float th[8])
{
    if (MIX && a.mix) return proposal_draw(a.tables[s], a.prop, a.key, i, d.series_id, a.prop_domain, th);
    prior_draw(a.key, i, d.series_id, a.domain, a.lo, a.width, th);
    return 1.0f;
}

// ----------------------------------------------------------------------------
// setup: log2(1 + O) table of all series
// ----------------------------------------------------------------------------
__global__ void k_batch_obs(const int32_t* const* obs, const SeriesDesc* desc, int m, float* table)
{
    const int s = blockIdx.x;
    if (s >= m) return;
    const SeriesDesc d = desc[s];
    for (int q = threadIdx.x; q < 3 * d.T; q += blockDim.x)
        table[d.obs_off + q] = (float)(log1p((double)obs[s][q]) * 1.44269504088896340736);
}

__global__ void k_batch_init(BatchArgs a)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.m) {
        SeriesState z{};
        z.target = a.target0;
        a.state[s] = z;
    }
}

// after a finalisation that kept fewer than Q rows of some series (float64
// decisions of band rows took more accepts away than the margin covered):
// raise their targets so that the next rounds continue their streams, by the
// shortfall over the series' observed ratio of kept rows to float32 accepts
// (at least 1/16), and the margin
__global__ void k_batch_retarget(BatchArgs a, const int64_t* count, int32_t margin)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.m) {
        SeriesState& st = a.state[s];
        const int64_t c = count[s];
        if (c >= 0 && c < a.quota && st.next < a.max_samples) {
            const double kept = (double)(c > 1 ? c : 1);
            double per = st.acc > 0 ? (double)st.acc / kept : 1.0;  // float32 accepts per kept row
            per = per < 1.0 ? 1.0 : (per > 16.0 ? 16.0 : per);
            st.target = st.acc + (int32_t)ceil((double)(a.quota - c) * per) + margin;
        }
    }
}

// truncated-mixture table of each series' proposal row: one workgroup per
// series, one thread per (component, dimension)
__global__ __launch_bounds__(64) void k_batch_tables(const float* mix, ProposalBox p, MixTable* tables)
{
    const int s = blockIdx.x;
    const float* o = mix + (int64_t)s * MIX_OUT;
    MixTable& t = tables[s];
    mix_table_entry(o, p, threadIdx.x / MIX_D, threadIdx.x % MIX_D, t);
    __syncthreads();
    if (threadIdx.x == 0) mix_table_finish(o, t);
}

// ----------------------------------------------------------------------------
// plan of one round (one workgroup of 256 threads, one series per thread)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(BT_MAX_SERIES) void k_batch_plan(BatchArgs a)
{
    __shared__ int wave_cnt[BT_MAX_SERIES / 64];
    __shared__ int chunk_wave[BT_MAX_SERIES / 64];
    // thread t plans series order[t]: chunks are laid out longest horizon
    // first, so every wave ends its share of a round on short trajectories
    const int tid = threadIdx.x;
    const int s = tid < a.m ? a.order[tid] : tid;
    const int lane = tid & 63, wave = tid >> 6;
    const int p = a.round;
    bool active = false;
    int64_t next = 0, done = 0, inflight = 0;
    int32_t cand_f = 0, acc_f = 0, target = 0;
    if (tid < a.m) {
        SeriesState& st = a.state[s];
        if (p >= 2) {
            // round p - 2 has finished (this plan runs after it): fold its counts
            const int f = (p - 2) % BT_SLOTS;
            st.acc_f += st.rc_acc[f];
            st.cand_f += st.rc_cand[f];
            st.done += st.n_slot[f];
            st.rc_acc[f] = 0;
            st.rc_cand[f] = 0;
            st.n_slot[f] = 0;
        }
        next = st.next;
        done = st.done;
        cand_f = st.cand_f;
        acc_f = st.acc_f;
        target = st.target;
        inflight = p >= 1 ? st.n_slot[(p - 1) % BT_SLOTS] : 0;  // round p - 1 may still run
        active = acc_f < target && next < a.max_samples;
    }
    const uint64_t bal = __ballot(active);
    const int rank_w = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(bal);
    __syncthreads();
    int before = 0, n_active = 0;
    for (int w = 0; w < BT_MAX_SERIES / 64; ++w) {
        if (w < wave) before += wave_cnt[w];
        n_active += wave_cnt[w];
    }
    const int rank = before + rank_w;
    int64_t n_s = 0;
    if (active) {
        const int64_t per = a.round_size / n_active;
        const int64_t rem = a.round_size % n_active;
        n_s = per + (rank < rem ? 1 : 0);
        if (n_s > a.max_samples - next) n_s = a.max_samples - next;
        // keep the expected candidates of the running round and this one
        // together within half the free capacity, at an upper bound of the
        // candidate rate of the finished rounds: (sqrt(c + 1) + 2)^2 for c
        // candidates, about four Poisson standard deviations above the count,
        // so that a round sized from the few candidates of a short first
        // round cannot overrun the capacity when they undercount the rate
        // (the schedule never changes which samples are accepted, only how
        // many rounds it takes)
        if (done > 0) {
            const double cu = sqrt((double)cand_f + 1.0) + 2.0;
            const double rate = cu * cu / (double)done;
            const double half = 0.5 * (double)((int64_t)a.cand_cap - cand_f) - rate * (double)inflight;
            int64_t lim = half > 0.0 ? (int64_t)(half / rate) : 0;
            if (lim < 64) lim = 64;
            if (n_s > lim) n_s = lim;
            // and no more samples than the target still needs: the running
            // round's samples and this round's must bring the float32
            // accepts to the target at a lower bound of their rate,
            // (sqrt(c) - 1)^2 per finished sample for c accepts (about two
            // Poisson standard deviations below the count). Without this, a
            // series' last rounds get a full share of the round, and the two
            // rounds planned before its count is known simulate samples past
            // its quota's last accept.
            if (acc_f >= 4) {
                const double cl = sqrt((double)acc_f) - 1.0;
                const double rlo = cl * cl / (double)done;
                const double left = (double)(target - acc_f) - rlo * (double)inflight;
                const int64_t need = left > 0.0 ? (int64_t)(left / rlo) + 64 : 64;
                if (n_s > need) n_s = need;
            }
        } else {
            // no finished round yet: every sample assigned so far may be a
            // candidate, so the series' samples stay within the capacity,
            // which no acceptance rate can overflow
            const int64_t left = (int64_t)a.cand_cap - next;
            if (n_s > left) n_s = left > 0 ? left : 0;
        }
    }
    const int chunks = (int)((n_s + 63) / 64);
    // exclusive scan of chunk counts in series order
    int incl = chunks;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) chunk_wave[wave] = incl;
    __syncthreads();
    int cbase = 0, ctot = 0;
    for (int w = 0; w < BT_MAX_SERIES / 64; ++w) {
        if (w < wave) cbase += chunk_wave[w];
        ctot += chunk_wave[w];
    }
    const int c0 = cbase + incl - chunks;
    RoundTable* t = a.table;
    if (active) {
        t->s[rank] = s;
        t->n[rank] = (int32_t)n_s;
        t->first[rank] = next;
        t->chunk0[rank] = c0;
        a.state[s].next = next + n_s;
    }
    if (tid < a.m) a.state[s].n_slot[p % BT_SLOTS] = n_s;
    if (tid == 0) {
        t->n_active = n_active;
        t->total_chunks = ctot;
        t->chunk0[n_active] = ctot;
        t->done = n_active == 0 ? 1 : 0;
    }
}

// ----------------------------------------------------------------------------
// one round: persistent grid with lane refill and per-lane series
// ----------------------------------------------------------------------------
struct alignas(16) BSlot {
    float a0, al, n, be, ga, de, bh;
    int32_t i0;
    uint32_t c1base, g3, h3, f3;  // per-sample part of Philox rounds 1-3
    int64_t i;                    // sample index
    int32_t series;               // index into desc, -1 = no sample
    int32_t pad;
};

struct BLane {
    State s;
    RatesF r;
    PhiloxDays ph;
    int64_t i;
    int32_t t;  // the day the slot simulates next; 0: no sample (idle)
    int32_t T, obs_off, series;
    float invP, exit2;
    uint32_t b1;
    float acc;
};

template <int SPL, bool MIX>
__global__ __launch_bounds__(1024 / SPL) void k_batch_round(BatchArgs a)
{
    extern __shared__ float lds_b[];
    __shared__ RoundTable tab_sh;  // copied once per workgroup
    const int nwaves_blk = blockDim.x >> 6;
    SeriesDesc* desc_sh = reinterpret_cast<SeriesDesc*>(lds_b);
    // the observed rows stay in global memory (read through the caches): in
    // LDS they would take 12 B per day of every series and leave room for
    // one workgroup per CU
    BSlot* ring_all = reinterpret_cast<BSlot*>(desc_sh + a.m);

    // stage the round table and the series descriptors
    {
        const int32_t* src = reinterpret_cast<const int32_t*>(a.table);
        int32_t* dst = reinterpret_cast<int32_t*>(&tab_sh);
        for (int q = threadIdx.x; q < (int)(sizeof(RoundTable) / 4); q += blockDim.x) dst[q] = src[q];
        const int32_t* dsrc = reinterpret_cast<const int32_t*>(a.desc);
        int32_t* ddst = reinterpret_cast<int32_t*>(desc_sh);
        for (int q = threadIdx.x; q < a.m * (int)(sizeof(SeriesDesc) / 4); q += blockDim.x)
            ddst[q] = dsrc[q];
    }
    __syncthreads();
    const int C = tab_sh.total_chunks;
    const int na = tab_sh.n_active;
    if (C == 0) return;

    const int lane = threadIdx.x & 63;
    // the wavefront index is uniform over the wave: kept scalar, so is the
    // queue arithmetic derived from it
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    BSlot* ring = ring_all + wv * BT_RING;
    const int64_t wg = (int64_t)blockIdx.x * nwaves_blk + wv;
    const int64_t nw = (int64_t)gridDim.x * nwaves_blk;
    if (wg >= C) return;
    const int64_t J = (C - 1 - wg) / nw + 1;  // chunks of this wave
    const int64_t Q = J << 6;

    // fill the ring with chunk j of this wave (all 64 lanes, one sample each)
    auto fill = [&](int64_t j) {
        const int c = (int)(wg + j * nw);
        int lo = 0, hi = na - 1;  // the active slot r with chunk0[r] <= c < chunk0[r+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab_sh.chunk0[mid] <= c) lo = mid; else hi = mid - 1;
        }
        const int r = lo;
        const int s = tab_sh.s[r];
        const int64_t local = (int64_t)(c - tab_sh.chunk0[r]) * 64 + lane;
        BSlot sl;
        if (local < tab_sh.n[r]) {
            const SeriesDesc& d = desc_sh[s];
            const int64_t i = tab_sh.first[r] + local;
            float th[8];
            (void)batch_theta<MIX>(a, s, d, (uint64_t)i, th);
            const Theta tt = theta_from(th);
            const RatesF rr = rates_f32(tt);
            const State s0 = init_state(tt.ka, d.P, d.A0, d.R0, d.D0);
            sl.a0 = rr.a0; sl.al = rr.al; sl.n = rr.n; sl.be = rr.be;
            sl.ga = rr.ga; sl.de = rr.de; sl.bh = rr.bh; sl.i0 = s0.I;
            PhiloxDays ph;
            ph.begin((uint64_t)i, d.u0, a.key);
            sl.c1base = ph.c1base; sl.g3 = ph.g3; sl.h3 = ph.h3; sl.f3 = ph.f3;
            sl.series = s;
            sl.i = i;
        } else {
            sl.series = -1;
            sl.i = 0;
        }
        sl.pad = 0;
        ring[lane] = sl;
    };

    int64_t q_base = 0;      // next queue position
    int64_t filled_j = -1;   // chunk currently in the ring
    BLane L[SPL];
#pragma unroll
    for (int k = 0; k < SPL; ++k) L[k].t = 0;
    uint32_t days_done = 0;

    while (true) {
        // refill every idle slot from the wave queue, in queue order; the ring
        // holds one chunk, so a refill may span the end of one chunk and the
        // start of the next
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            uint64_t m = __ballot(L[k].t == 0);
            if (__popcll(m) < a.refill_min) continue;  // let a few more lanes finish first
            while (m != 0ull && q_base < Q) {
                const int64_t j = q_base >> 6;
                if (j != filled_j) {
                    fill(j);
                    filled_j = j;
                }
                const int avail = 64 - (int)(q_base & 63);
                const bool inm = (m >> lane) & 1ull;
                // lanes of m below this one
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const bool take = inm && rank < avail;
                if (take) {
                    const BSlot sl = ring[(q_base & 63) + rank];
                    if (sl.series >= 0) {
                        const SeriesDesc& d = desc_sh[sl.series];
                        BLane& l = L[k];
                        l.r = RatesF{sl.a0, sl.al, sl.n, sl.be, sl.ga, sl.de, sl.bh};
                        l.s.A = d.A0; l.s.R = d.R0; l.s.D = d.D0; l.s.Ru = 0;
                        l.s.I = sl.i0;
                        l.s.S = d.room - sl.i0;
                        l.ph.c1base = sl.c1base; l.ph.g3 = sl.g3; l.ph.h3 = sl.h3; l.ph.f3 = sl.f3;
                        l.i = sl.i;
                        l.t = 1;
                        l.T = d.T;
                        l.obs_off = d.obs_off;
                        l.series = sl.series;
                        l.invP = d.invP;
                        l.exit2 = d.exit2;
                        l.b1 = d.b1;
                        l.acc = 0.0f;
                    }
                }
                const int cnt = __popcll(m);
                q_base += cnt < avail ? cnt : avail;
                m = __ballot(inm && !take);  // lanes still without a position
            }
        }
        bool any = false;
#pragma unroll
        for (int k = 0; k < SPL; ++k) any |= L[k].t != 0;
        // a refill can land every idle lane on the unused tail of a series'
        // last chunk; the wave ends only when the queue is exhausted too
        if (__ballot(any) == 0ull && q_base >= Q) break;

#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            BLane& l = L[k];
            if (l.t == 0) continue;
            const int t = l.t;
            const uint4 w = l.ph.day(((uint32_t)t << 8) | (a.domain << 4), l.b1, a.key);
            Noise32 z;
            normals_f32(w, a.nc, z);
            day_step_f32<0>(l.s, l.r, l.invP, z);
            const int32_t X[3] = {l.s.A, l.s.R, l.s.D};
            const float* ob = a.obs_table + l.obs_off + t - 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float d = log2p1_count_f32(X[c]) - ob[c * l.T];
                l.acc = fmaf(d, d, l.acc);
            }
            ++days_done;
            const bool exited = l.acc > l.exit2;
            if (exited || t == l.T) {
                if (!exited) {
                    const float dd = finish_distance_f32(l.acc, 0.693147180559945309417f);
                    const SeriesDesc& ds = desc_sh[l.series];
                    if (dd <= ds.eps_hi) {
                        SeriesState& st = a.state[l.series];
                        const int pos = atomicAdd(&st.cand, 1);
                        atomicAdd(&st.rc_cand[a.round % BT_SLOTS], 1);
                        if (pos < a.cand_cap) {
                            a.cand_idx[(int64_t)l.series * a.cand_cap + pos] = l.i;
                            a.cand_dist[(int64_t)l.series * a.cand_cap + pos] = dd;
                        }
                        if (dd <= ds.eps_cnt) {
                            atomicAdd(&st.acc, 1);
                            atomicAdd(&st.rc_acc[a.round % BT_SLOTS], 1);
                        }
                    }
                }
                l.t = 0;
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

// 1 once every series has reached its target of float32 accepts or used its
// maximum
__global__ __launch_bounds__(BT_MAX_SERIES) void k_batch_flag(BatchArgs a)
{
    __shared__ int open;
    if (threadIdx.x == 0) open = 0;
    __syncthreads();
    const int s = threadIdx.x;
    if (s < a.m && a.state[s].acc < a.state[s].target && a.state[s].next < a.max_samples)
        atomicAdd(&open, 1);
    __syncthreads();
    if (threadIdx.x == 0) *a.flag_dev = open == 0 ? 1 : 0;
}

// ----------------------------------------------------------------------------
// finalisation: one workgroup per series
// ----------------------------------------------------------------------------
struct FinalArgs {
    BatchArgs b;
    const int32_t* const* obs;  // raw observed counts per series (float64 decision)
    float band_w;
    int64_t* out_idx;    // [m][quota]
    float* out_theta;    // [m][quota][8]
    float* out_w;        // [m][quota] importance weights, or null
    float* out_dist;     // [m][quota]
    int64_t* out_count;  // [m]
    int64_t* out_used;   // [m] samples consumed
    int32_t* out_rechecked;
    int32_t* band_n;     // [m] band rows of each series (zeroed before k_band_collect)
    int32_t* band_q;     // [m][cand_cap] their positions in the candidate list
    int32_t* band_next;  // chunk counter of k_batch_band (zeroed with band_n)
    int32_t* band_from;  // [m] candidates decided by earlier finalisations (zeroed once)
};

// bitonic sort of (idx, dist) pairs in LDS, ascending by idx. Each step
// compares element t with t ^ j; the threads walk the n_pow2 / 2 pairs
// directly (pair i gives t by inserting a zero at bit log2 j), so no lane
// idles on the upper element of a pair.
__device__ void bitonic_sort(int64_t* key, float* val, int n_pow2)
{
    const int half = n_pow2 >> 1;
    for (int k = 2; k <= n_pow2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < half; i += blockDim.x) {
                const int t = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int p = t | j;
                const bool up = (t & k) == 0;
                const int64_t a = key[t], b = key[p];
                if ((a > b) == up) {
                    key[t] = b; key[p] = a;
                    const float v = val[t]; val[t] = val[p]; val[p] = v;
                }
            }
            __syncthreads();
        }
    }
}

// Float64 decision of the band rows (candidates with eps (1 - w) < d <=
// eps (1 + w)), in two kernels. k_band_collect lists each series' band rows
// (positions in its candidate list, in any order: each row is decided on its
// own). k_batch_band is a persistent grid of one-wavefront workgroups that
// take chunks of up to rows_max rows of one series from a global counter and
// simulate them in float64 side by side (simulate_rows_f64_wave: each row's
// distance is the double simulate_one_f64 gives), so every walk but the last
// of a series is full and no wavefront waits on another's series. A decided
// row keeps its float64 distance (as float); a rejected one gets idx
// INT64_MAX, which sorts it last.
constexpr int COLLECT_GROUPS = 4;  // workgroups of 256 per series in the collection

__global__ __launch_bounds__(256) void k_band_collect(FinalArgs f)
{
    const BatchArgs& a = f.b;
    const int s = blockIdx.x / COLLECT_GROUPS, g = blockIdx.x % COLLECT_GROUPS;
    const int cand = a.state[s].cand;
    const int n = cand < a.cand_cap ? cand : a.cand_cap;
    const int q0 = f.band_from[s];  // earlier finalisations decided the rows before q0
    const float lo = a.desc[s].eps_lo;
    const float* cdist = a.cand_dist + (int64_t)s * a.cand_cap;
    int32_t* bq = f.band_q + (int64_t)s * a.cand_cap;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int base = q0 + (g * 4 + (int)(threadIdx.x >> 6)) * 64; base < n; base += COLLECT_GROUPS * 256) {
        const int q = base + lane;
        const bool inb = q < n && cdist[q] > lo;
        const uint64_t m = __ballot(inb);
        if (m == 0ull) continue;
        int pos = 0;
        if (lane == 0) pos = atomicAdd(&f.band_n[s], __popcll(m));
        pos = __shfl(pos, 0, 64);
        if (inb) bq[pos + __popcll(m & below)] = q;
    }
}

__global__ __launch_bounds__(64) void k_batch_band(FinalArgs f, int rows_max, int max_T)
{
    extern __shared__ double lds_band[];
    __shared__ int pre[BT_MAX_SERIES + 1];  // first chunk of each series, in planning order
    const BatchArgs& a = f.b;
    const int lane = threadIdx.x;
    // chunks of series order[j]: ceil(band_n / rows_max), laid out in the
    // planning order (longest horizon first), so that the longest walks are
    // taken first and the short ones fill in around them
    int total = 0;
    for (int b0 = 0; b0 < a.m; b0 += 64) {
        const int j = b0 + lane;
        const int c = j < a.m ? (f.band_n[a.order[j]] + rows_max - 1) / rows_max : 0;
        int incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (j < a.m) pre[j + 1] = total + incl;
        total += __shfl(incl, 63, 64);
    }
    if (lane == 0) pre[0] = 0;
    __syncthreads();
    if (total == 0) return;
    double* lobs = lds_band;
    double* zs = lobs + 3 * max_T;
    uint64_t* rix = reinterpret_cast<uint64_t*>(zs + (size_t)5 * ROW_WINDOW * rows_max);
    int32_t* rq = reinterpret_cast<int32_t*>(rix + rows_max);
    RowWalk* rw = reinterpret_cast<RowWalk*>(rq + 2 * rows_max);  // rq padded to 8 B per row
    int32_t* xs = reinterpret_cast<int32_t*>(rw + rows_max);
    float* rth = reinterpret_cast<float*>(xs + (size_t)3 * ROW_WINDOW * rows_max);
    int staged = -1;
    for (;;) {
        int c = 0;
        if (lane == 0) c = atomicAdd(f.band_next, 1);
        c = __shfl(c, 0, 64);
        if (c >= total) break;
        // the series whose chunks hold c: pre[j] <= c < pre[j + 1], s = order[j]
        int lo = 0, hi = a.m;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= c) lo = mid;
            else hi = mid;
        }
        const int s = a.order[lo];
        const SeriesDesc d = a.desc[s];
        const int j0 = (c - pre[lo]) * rows_max;
        const int nb = f.band_n[s];
        const int nr = nb - j0 < rows_max ? nb - j0 : rows_max;
        int64_t* cidx = a.cand_idx + (int64_t)s * a.cand_cap;
        float* cdist = a.cand_dist + (int64_t)s * a.cand_cap;
        if (staged != s) {
            stage_obs_f64<0>(f.obs[s], d.T, lobs);
            staged = s;
        }
        if (lane < nr) {
            const int q = f.band_q[(int64_t)s * a.cand_cap + j0 + lane];
            const int64_t k = cidx[q];
            rq[lane] = q;
            rix[lane] = (uint64_t)k;
            float th[8];
            (void)batch_theta(a, s, d, (uint64_t)k, th);
#pragma unroll
            for (int j = 0; j < 8; ++j) rth[8 * lane + j] = th[j];
        }
        __syncthreads();
        const double d64 = simulate_rows_f64_wave<0, 0>(nr, rth, rix, a.key, d.series_id, a.domain, d.P,
                                                       d.A0, d.R0, d.D0, d.T, (double)a.scale, lobs, zs,
                                                       xs, rw);
        if (lane < nr) {
            const int q = rq[lane];
            cdist[q] = (float)d64;
            if (!(d64 <= (double)d.eps)) cidx[q] = INT64_MAX;
        }
        if (lane == 0 && f.out_rechecked) atomicAdd(&f.out_rechecked[s], nr);
        __syncthreads();  // the observed rows and row slots are refilled next
    }
}

static size_t band_lds_bytes(int maxT, int R)
{
    return sizeof(double) * 3 * (size_t)maxT +
           (size_t)R * (sizeof(double) * 5 * ROW_WINDOW + sizeof(uint64_t) + 2 * sizeof(int32_t) +
                        sizeof(RowWalk) + sizeof(int32_t) * 3 * ROW_WINDOW + sizeof(float) * 8);
}

// Finalisation: one workgroup per series sorts its candidates by index and
// writes the first quota kept rows. The sort is bound by LDS latency, so the
// workgroup is as large as allowed (16 wavefronts; 82 VGPRs, no spills).
constexpr int FINAL_BLOCK = 1024;

__global__ __launch_bounds__(FINAL_BLOCK) void k_batch_final(FinalArgs f)
{
    extern __shared__ unsigned char lds_f8[];
    const BatchArgs& a = f.b;
    const int s = blockIdx.x;
    const SeriesDesc d = a.desc[s];
    const int cand = a.state[s].cand;
    int n = cand < a.cand_cap ? cand : a.cand_cap;
    int npow = 1;
    while (npow < n) npow <<= 1;
    int64_t* key = reinterpret_cast<int64_t*>(lds_f8);
    float* val = reinterpret_cast<float*>(key + npow);
    __shared__ int nkeep;
    if (threadIdx.x == 0) nkeep = 0;
    // the band rows were decided in float64 by k_batch_band (rejected: idx INT64_MAX)
    for (int q = threadIdx.x; q < npow; q += blockDim.x) {
        int64_t k = INT64_MAX;
        float v = INFINITY;
        if (q < n) {
            k = a.cand_idx[(int64_t)s * a.cand_cap + q];
            v = a.cand_dist[(int64_t)s * a.cand_cap + q];
        }
        key[q] = k;
        val[q] = v;
    }
    __syncthreads();
    bitonic_sort(key, val, npow);
    for (int q = threadIdx.x; q < npow && q < a.quota; q += blockDim.x) {
        if (key[q] != INT64_MAX) {
            f.out_idx[(int64_t)s * a.quota + q] = key[q];
            f.out_dist[(int64_t)s * a.quota + q] = val[q];
            float th[8];
            const float w = batch_theta(a, s, d, (uint64_t)key[q], th);
#pragma unroll
            for (int j = 0; j < 8; ++j) f.out_theta[((int64_t)s * a.quota + q) * 8 + j] = th[j];
            if (f.out_w) f.out_w[(int64_t)s * a.quota + q] = w;
            atomicAdd(&nkeep, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        f.out_count[s] = cand > a.cand_cap ? -(int64_t)cand : (int64_t)nkeep;
        f.out_used[s] = a.state[s].next;
        f.band_from[s] = n;
    }
}

// Float64 mean and covariance of each series' accepted theta: one workgroup
// per series, fixed reduction order.

// V sums at once: each is reduced by a butterfly within the wavefront, then
// over the wavefronts in order (a fixed order); red holds [waves][V]
template <int V>
__device__ void block_sum_f64_v(double (&v)[V], double* red)
{
#pragma unroll
    for (int i = 0; i < V; ++i) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < V; ++i) red[wave * V + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w * V + i];
        v[i] = t;
    }
}

__global__ __launch_bounds__(256) void k_batch_moments(const float* theta, const float* weight,
                                                       const int64_t* count, int quota, double* mean,
                                                       double* cov)
{
    __shared__ double red[4 * 36];
    const int s = blockIdx.x;
    const int64_t n = count[s] > 0 ? (count[s] < quota ? count[s] : quota) : 0;
    const float* th = theta + (int64_t)s * quota * 8;
    const float* w = weight ? weight + (int64_t)s * quota : nullptr;
    // unweighted: mean and the unbiased (n - 1) covariance; weighted: sum w theta / V1
    // and sum w (theta - mean)(theta - mean)^T / (V1 - V2 / V1). One pass over
    // the rows per stage (weights, means, centred products), every sum of a
    // stage reduced together.
    double v1 = (double)n, v2 = (double)n;
    if (w) {
        double a[2] = {0.0, 0.0};
        for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
            const double x = (double)w[r];
            a[0] += x;
            a[1] += x * x;
        }
        block_sum_f64_v(a, red);
        v1 = a[0];
        v2 = a[1];
    }
    double mu[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) mu[j] = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double x = w ? (double)w[r] : 1.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) mu[j] += x * (double)th[8 * r + j];
    }
    block_sum_f64_v(mu, red);
#pragma unroll
    for (int j = 0; j < 8; ++j) mu[j] /= v1;
    const double denom = w ? v1 - v2 / v1 : (double)(n - 1);
    double cv[36];
#pragma unroll
    for (int q = 0; q < 36; ++q) cv[q] = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double x = w ? (double)w[r] : 1.0;
        double d[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) d[j] = (double)th[8 * r + j] - mu[j];
        int q = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int l = j; l < 8; ++l) cv[q++] += x * (d[j] * d[l]);
    }
    block_sum_f64_v(cv, red);
    if (threadIdx.x == 0) {
        int q = 0;
        for (int j = 0; j < 8; ++j)
            for (int l = j; l < 8; ++l) {
                const double c = cv[q++] / denom;
                cov[(int64_t)s * 64 + 8 * j + l] = c;
                cov[(int64_t)s * 64 + 8 * l + j] = c;
            }
        for (int j = 0; j < 8; ++j) mean[(int64_t)s * 8 + j] = n > 0 ? mu[j] : NAN;
    }
}

static size_t batch_lds_bytes(int m, int obs_words, int block)
{
    (void)obs_words;  // the observed rows are read from global memory
    return sizeof(SeriesDesc) * (size_t)m + sizeof(BSlot) * BT_RING * (size_t)(block / 64);
}

}  // namespace abc

using namespace abc;

namespace {

template <int SPL>
void launch_round(const BatchArgs& a, unsigned grid, int block, size_t lds, hipStream_t s)
{
    if (a.mix)
        hipLaunchKernelGGL((k_batch_round<SPL, true>), dim3(grid), dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL((k_batch_round<SPL, false>), dim3(grid), dim3(block), lds, s, a);
}

}  // namespace

static abc_status batch_run(const abc_batch_series* series, int32_t m, const abc_prior* prior,
                            const abc_model* model, uint64_t seed, uint32_t domain, int32_t quota,
                            int64_t round_size, int64_t max_samples, float band_w,
                            int32_t rounds_per_graph, int32_t cand_capacity,
                            const abc_batch_proposal* prop, int64_t* out_idx, float* out_theta,
                            float* out_w, float* out_dist, int64_t* out_count, int64_t* out_used,
                            double* out_mean, double* out_cov, abc_batch_stats* stats, void* stream)
{
    abc_status rc;
    ABC_REQUIRE(series != nullptr && m >= 1 && m <= BT_MAX_SERIES, "need 1 <= m <= %d series", BT_MAX_SERIES);
    if ((rc = check_model(model))) return rc;
    ABC_REQUIRE((model->flags & (ABC_FP64 | ABC_KAHAN | ABC_NOISE_LITERAL | ABC_DIST_RAW)) == 0,
                "the batched path runs the default model in float32 (flags must be 0)");
    ABC_REQUIRE(domain <= 15u, "domain > 15");
    ABC_REQUIRE(quota >= 1 && quota <= 4096, "quota must be in [1, 4096]");
    ABC_REQUIRE(round_size >= 64, "round_size < 64");
    ABC_REQUIRE(max_samples >= 1, "max_samples < 1");
    ABC_REQUIRE(isfinite(band_w) && band_w >= 0.0f && band_w < 1.0f, "band_w must be in [0, 1)");
    ABC_REQUIRE(rounds_per_graph >= 1 && rounds_per_graph <= 64, "rounds_per_graph in [1, 64]");
    ABC_REQUIRE(out_idx && out_theta && out_dist && out_count && out_used && out_mean && out_cov,
                "NULL output pointer");
    ABC_REQUIRE(cand_capacity == 0 || (cand_capacity >= quota && cand_capacity <= 16384),
                "cand_capacity must be 0 (max(4 quota, 256)) or in [quota, 16384]");
    float lo[8], width[8];
    if ((rc = prior_lo_width(prior, lo, width))) return rc;
    for (int k = 0; k < 8; ++k) ABC_REQUIRE(prior->lo[k] >= 0.0f, "prior lo[%d] < 0", k);
    if (prop) {
        ABC_REQUIRE(prop->mix != nullptr && out_w != nullptr, "proposal rows and out_w are required");
        ABC_REQUIRE(prop->lambda >= 0.0f && prop->lambda <= 1.0f, "lambda must be in [0, 1]");
        ABC_REQUIRE(isfinite(prop->inflate) && prop->inflate >= 1.0f && prop->inflate <= 100.0f,
                    "inflate must be in [1, 100]");
        ABC_REQUIRE(prop->domain <= 15u, "proposal domain > 15");
        // theta's Philox words (day 1 of the proposal domain) must not be the
        // simulation's day-1 noise words: a sample would be correlated with
        // its own trajectory
        ABC_REQUIRE(prop->domain != domain, "proposal domain %u equals the simulation domain",
                    prop->domain);
    }

    // host-side series descriptors
    std::vector<SeriesDesc> desc(m);
    std::vector<const int32_t*> obs_ptr(m);
    int obs_words = 0, maxT = 0;
    const Key key = make_key(seed);
    for (int s = 0; s < m; ++s) {
        const abc_batch_series& b = series[s];
        abc_series ser{b.P, b.A0, b.R0, b.D0, b.T, b.obs};
        if ((rc = check_series(&ser, true))) return set_error(rc, "series %d: %s", s, abc_last_error());
        ABC_REQUIRE(isfinite(b.eps) && b.eps >= 0.0f, "series %d: eps must be finite and >= 0", s);
        SeriesDesc& d = desc[s];
        d.T = b.T; d.P = (int32_t)b.P; d.A0 = b.A0; d.R0 = b.R0; d.D0 = b.D0;
        d.obs_off = obs_words;
        d.room = (int32_t)b.P - (b.A0 + b.R0 + b.D0);
        d.series_id = b.series;
        d.invP = 1.0f / (float)b.P;
        const double hi = (double)b.eps * (1.0 + (double)band_w);
        d.eps_hi = (float)hi;
        d.eps_lo = (float)((double)b.eps * (1.0 - (double)band_w));
        d.eps = b.eps;
        d.eps_cnt = (float)((double)b.eps * (1.0 - BT_TIE));
        d.exit2 = (float)(hi * hi * 2.08136898100560809980 * (1.0 + 0x1p-18));
        const uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)b.series;
        d.u0 = (uint32_t)(p1 >> 32) ^ key.k0;
        d.b1 = (uint32_t)p1 ^ (key.k0 + PH_W0);
        obs_words += 3 * b.T;
        obs_ptr[s] = b.obs;
        if (b.T > maxT) maxT = b.T;
    }
    int32_t spl = 1, block = 1024, bpc = 1;
    abc_get_launch_config(&spl, &block, &bpc);
    if (spl != 1 && spl != 2 && spl != 4 && spl != 8)
        return set_error(ABC_EUNSUPPORTED, "the batched round kernel is built for 1, 2, 4 or 8 "
                         "samples per lane, not %d", spl);
    const int32_t refill_min = abc_get_refill_min();
    const size_t lds = batch_lds_bytes(m, obs_words, block);
    DeviceInfo info;
    if ((rc = device_info(&info))) return rc;
    const int num_cu = info.num_cu, max_lds = info.max_lds;
    const size_t static_lds = sizeof(RoundTable);
    if (lds + static_lds > (size_t)max_lds)
        return set_error(ABC_EUNSUPPORTED,
                         "batch needs %zu B of LDS per workgroup (> %d): split the series into groups",
                         lds + static_lds, max_lds);
    // default candidate rows: 4 quota, and never fewer than 256 so that a
    // small quota does not leave a one-chunk share able to overflow the list
    const int cand_default = 4 * quota > 256 ? 4 * quota : 256;
    {
        int np = 1;
        while (np < (cand_capacity ? cand_capacity : cand_default)) np <<= 1;
        const size_t lds_final = sizeof(int64_t) * np + sizeof(float) * (np + 1) + 16;
        if (lds_final > (size_t)max_lds)
            return set_error(ABC_EINVAL, "cand_capacity %d needs %zu B of LDS to sort (> %d)",
                             cand_capacity ? cand_capacity : cand_default, lds_final, max_lds);
    }
    const int per_cu = (int)(163840 / (lds + static_lds));
    const unsigned grid = (unsigned)num_cu * (unsigned)(per_cu < bpc ? (per_cu > 0 ? per_cu : 1) : bpc);
    const int cand_cap = cand_capacity ? cand_capacity : cand_default;
    int npow_cap = 1;
    while (npow_cap < cand_cap) npow_cap <<= 1;

    // Device buffers from the library's scratch arena on the caller's stream
    // (the call's own stream below starts after the caller's earlier work and
    // the caller's stream waits for it before the call returns, so the next
    // call on that stream reuses them safely); the completion flag lives in
    // the arena's pinned host buffer of the same stream.
    hipStream_t user = as_stream(stream);
    struct Carve {
        size_t off = 0;
        size_t take(size_t bytes) { const size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; }
    } carve;
    const size_t o_desc = carve.take(sizeof(SeriesDesc) * m);
    const size_t o_state = carve.take(sizeof(SeriesState) * m);
    constexpr int BT_EVR = 8;  // events and completion flags in a ring over the rounds
    const size_t o_table = carve.take(2 * sizeof(RoundTable));
    const size_t o_obs = carve.take(sizeof(float) * (size_t)obs_words);
    const size_t o_ptrs = carve.take(sizeof(const int32_t*) * m);
    const size_t o_cidx = carve.take(sizeof(int64_t) * (size_t)m * cand_cap);
    const size_t o_cdist = carve.take(sizeof(float) * (size_t)m * cand_cap);
    const size_t o_flag = carve.take(sizeof(int32_t) * BT_EVR);
    const size_t o_days = carve.take(sizeof(unsigned long long));
    const size_t o_order = carve.take(sizeof(int32_t) * m);
    const size_t o_mixtab = carve.take(prop ? sizeof(MixTable) * m : 0);
    // rechecked, band_n, chunk counter (cleared by every finalisation), band_from
    const size_t o_re = carve.take(sizeof(int32_t) * (3 * (size_t)m + 1));
    const size_t o_bq = carve.take(sizeof(int32_t) * (size_t)m * cand_cap);
    void* arena = nullptr;
    if ((rc = stream_scratch(user, carve.off, &arena, SCRATCH_BATCH))) return rc;
    char* base = static_cast<char*>(arena);
    struct View { void* p; } b_desc{base + o_desc}, b_state{base + o_state}, b_table{base + o_table},
        b_obs{base + o_obs}, b_ptrs{base + o_ptrs}, b_cidx{base + o_cidx}, b_cdist{base + o_cdist},
        b_flag{base + o_flag}, b_days{base + o_days}, b_order{base + o_order}, b_mixtab{base + o_mixtab},
        b_re{base + o_re}, b_bq{base + o_bq};
    int32_t* flag_host = nullptr;
    if ((rc = stream_pinned(user, sizeof(int32_t) * BT_EVR, reinterpret_cast<void**>(&flag_host)))) return rc;

    hipStream_t s;
    ABC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamFree {
        hipStream_t s;
        ~StreamFree() { (void)hipStreamDestroy(s); }
    } stream_free{s};
    hipEvent_t ev;
    ABC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    struct EventFree {
        hipEvent_t e;
        ~EventFree() { (void)hipEventDestroy(e); }
    } event_free{ev};
    ABC_HIP(hipEventRecord(ev, user));
    ABC_HIP(hipStreamWaitEvent(s, ev, 0));

    ABC_HIP(hipMemcpyAsync(b_desc.p, desc.data(), sizeof(SeriesDesc) * m, hipMemcpyHostToDevice, s));
    ABC_HIP(hipMemcpyAsync(b_ptrs.p, obs_ptr.data(), sizeof(const int32_t*) * m, hipMemcpyHostToDevice, s));
    std::vector<int32_t> order(m);
    for (int q = 0; q < m; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return series[x].T > series[y].T; });
    ABC_HIP(hipMemcpyAsync(b_order.p, order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    ABC_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope with this call

    BatchArgs a{};
    a.m = m;
    a.quota = quota;
    a.target0 = std::max(1, quota + (g_batch_margin != 0 ? g_batch_margin : std::max(4, quota / 256)));
    a.round_size = round_size;
    a.max_samples = max_samples;
    a.cand_cap = cand_cap;
    a.obs_words = obs_words;
    a.key = key;
    a.domain = domain;
    for (int k = 0; k < 8; ++k) { a.lo[k] = lo[k]; a.width[k] = width[k]; }
    a.desc = reinterpret_cast<const SeriesDesc*>(b_desc.p);
    a.order = reinterpret_cast<const int32_t*>(b_order.p);
    a.state = reinterpret_cast<SeriesState*>(b_state.p);
    a.table = reinterpret_cast<RoundTable*>(b_table.p);
    a.obs_table = reinterpret_cast<const float*>(b_obs.p);
    a.cand_idx = reinterpret_cast<int64_t*>(b_cidx.p);
    a.cand_dist = reinterpret_cast<float*>(b_cdist.p);
    a.flag_dev = reinterpret_cast<int32_t*>(b_flag.p);
    a.days = reinterpret_cast<unsigned long long*>(b_days.p);
    a.nc = -1.38629436111989061883f * model->noise_scale * model->noise_scale;
    a.scale = model->noise_scale;
    a.refill_min = refill_min;
    if (prop) {
        a.mix = prop->mix;
        for (int k = 0; k < 8; ++k) { a.prop.lo[k] = prior->lo[k]; a.prop.hi[k] = prior->hi[k]; }
        proposal_standardiser(a.prop.lo, a.prop.hi, a.prop.tc, a.prop.ts);
        a.prop.lambda = prop->lambda;
        a.prop.log_inflate = logf(prop->inflate);
        a.prop_domain = prop->domain;
        a.tables = reinterpret_cast<const MixTable*>(b_mixtab.p);
        hipLaunchKernelGGL(k_batch_tables, dim3(m), dim3(MIX_K * MIX_D), 0, s, a.mix, a.prop,
                           reinterpret_cast<MixTable*>(b_mixtab.p));
        if ((rc = check_launch("k_batch_tables"))) return rc;
    }

    hipLaunchKernelGGL(k_batch_obs, dim3(m), dim3(256), 0, s,
                       reinterpret_cast<const int32_t* const*>(b_ptrs.p), a.desc, m,
                       reinterpret_cast<float*>(b_obs.p));
    hipLaunchKernelGGL(k_batch_init, dim3((m + 255) / 256), dim3(256), 0, s, a);
    if ((rc = check_launch("k_batch setup"))) return rc;
    ABC_HIP(hipMemsetAsync(b_days.p, 0, sizeof(unsigned long long), s));
    ABC_HIP(hipMemsetAsync(b_re.p, 0, sizeof(int32_t) * (3 * (size_t)m + 1), s));

    // Rounds alternate between two streams; plan p runs on s after plan
    // p - 1 and after round p - 2, round p after plan p, so round p - 1 can
    // still be finishing its last trajectories while round p starts. A
    // completion flag (every series at quota or at max_samples, from the
    // counts of all finished samples) follows each round; the host reads the
    // flag of round p - L (L = rounds_per_graph, at least 2) after enqueueing
    // round p. A flag that says done was computed after round q finished,
    // possibly during round q + 1, so the counts were done by the end of
    // round q + 1 and plans from q + 3 on assign no samples: the rounds up to
    // q + 2 are all the result depends on, and with L >= 2 they have been
    // enqueued by then.
    hipStream_t rs[2] = {nullptr, nullptr};
    struct RoundStreams {
        hipStream_t* r;
        ~RoundStreams() { for (int k = 0; k < 2; ++k) if (r[k]) (void)hipStreamDestroy(r[k]); }
    } round_streams{rs};
    for (int k = 0; k < 2; ++k) ABC_HIP(hipStreamCreateWithFlags(&rs[k], hipStreamNonBlocking));
    hipEvent_t ev_plan[BT_EVR] = {}, ev_round[BT_EVR] = {};
    struct RoundEvents {
        hipEvent_t* a;
        hipEvent_t* b;
        ~RoundEvents() {
            for (int k = 0; k < BT_EVR; ++k) {
                if (a[k]) (void)hipEventDestroy(a[k]);
                if (b[k]) (void)hipEventDestroy(b[k]);
            }
        }
    } round_events{ev_plan, ev_round};
    for (int k = 0; k < BT_EVR; ++k) {
        ABC_HIP(hipEventCreateWithFlags(&ev_plan[k], hipEventDisableTiming));
        ABC_HIP(hipEventCreateWithFlags(&ev_round[k], hipEventDisableTiming));
    }
    RoundTable* tables = reinterpret_cast<RoundTable*>(b_table.p);
    int32_t* flags_dev = reinterpret_cast<int32_t*>(b_flag.p);
    for (int k = 0; k < BT_EVR; ++k) flag_host[k] = 0;
    const int L = rounds_per_graph < 2 ? 2 : (rounds_per_graph > BT_EVR - 2 ? BT_EVR - 2 : rounds_per_graph);
    const int64_t max_rounds =
        ((max_samples * (int64_t)m + round_size - 1) / round_size + 2) * 2 + 4;
    hipEvent_t t0, t1;
    ABC_HIP(hipEventCreate(&t0));
    ABC_HIP(hipEventCreate(&t1));
    struct TimerFree {
        hipEvent_t a, b;
        ~TimerFree() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } timer_free{t0, t1};
    ABC_HIP(hipEventRecord(t0, s));
    FinalArgs f{};
    f.b = a;
    f.obs = reinterpret_cast<const int32_t* const*>(b_ptrs.p);
    f.band_w = band_w;
    f.out_idx = out_idx;
    f.out_theta = out_theta;
    f.out_w = prop ? out_w : nullptr;
    f.out_dist = out_dist;
    f.out_count = out_count;
    f.out_used = out_used;
    f.out_rechecked = reinterpret_cast<int32_t*>(b_re.p);
    f.band_n = f.out_rechecked + m;
    f.band_next = f.band_n + m;
    f.band_from = f.band_next + 1;
    f.band_q = reinterpret_cast<int32_t*>(b_bq.p);
    const int npow = npow_cap;
    const size_t lds_f = sizeof(int64_t) * npow + sizeof(float) * (npow + 1) + 16;
    ABC_REQUIRE(lds_f <= (size_t)max_lds, "quota too large for the finalisation");
    const int band_rows = ROWS_PER_WAVE_MAX;
    const size_t lds_band = band_lds_bytes(maxT, band_rows);
    ABC_REQUIRE(lds_band <= (size_t)max_lds, "horizon too long for the band decision");
    // A series stops taking samples once its float32 accepts (d <= eps)
    // reach its target, first Q + margin. Float64 decisions of band rows can
    // take a few of those accepts away (and add others); a finalisation that
    // keeps fewer than Q rows of a series raises its target by the shortfall
    // and the margin, and the rounds continue its stream: each phase only
    // adds samples in index order, and the last finalisation decides every
    // candidate, so the rows kept are still the first Q accepts.
    const int32_t margin = std::max(4, quota / 256);  // of every later target
    int64_t rounds = 0, polls = 0, stop_at = -1, phase0 = 0, rechecked = 0;
    int32_t phases = 0;
    std::vector<int64_t> cnt(m), used_h(m);
    std::vector<int32_t> rech(m);
    float rounds_ms = 0.0f;
    for (;;) {
        const int64_t round_cap = rounds + max_rounds;
        while (rounds < round_cap && (stop_at < 0 || rounds <= stop_at)) {
            const int64_t p = rounds;
            const int e = (int)(p % BT_EVR);
            BatchArgs ap = a;
            ap.table = tables + (p & 1);
            ap.round = (int32_t)p;
            ap.flag_dev = flags_dev + e;
            if (p >= 2) ABC_HIP(hipStreamWaitEvent(s, ev_round[(p - 2) % BT_EVR], 0));
            hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(BT_MAX_SERIES), 0, s, ap);
            ABC_HIP(hipEventRecord(ev_plan[e], s));
            hipStream_t r = rs[p & 1];
            ABC_HIP(hipStreamWaitEvent(r, ev_plan[e], 0));
            switch (spl) {
            case 1: launch_round<1>(ap, grid, block, lds, r); break;
            case 2: launch_round<2>(ap, grid, block, lds, r); break;
            case 4: launch_round<4>(ap, grid, block, lds, r); break;
            case 8: launch_round<8>(ap, grid, block, lds, r); break;
            }
            hipLaunchKernelGGL(k_batch_flag, dim3(1), dim3(BT_MAX_SERIES), 0, r, ap);
            ABC_HIP(hipMemcpyAsync(flag_host + e, ap.flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, r));
            ABC_HIP(hipEventRecord(ev_round[e], r));
            if ((rc = check_launch("k_batch round"))) return rc;
            ++rounds;
            if (p >= phase0 + L && stop_at < 0) {
                const int64_t q = p - L;
                ABC_HIP(hipEventSynchronize(ev_round[q % BT_EVR]));
                ++polls;
                if (flag_host[q % BT_EVR]) stop_at = q + 2;
            }
        }
        // the last two rounds are on the two round streams
        for (int64_t q = rounds - 2; q < rounds; ++q)
            if (q >= 0) ABC_HIP(hipStreamWaitEvent(s, ev_round[q % BT_EVR], 0));
        ABC_HIP(hipEventRecord(t1, s));
        ABC_HIP(hipEventSynchronize(t1));
        ABC_HIP(hipEventElapsedTime(&rounds_ms, t0, t1));

        ABC_HIP(hipMemsetAsync(b_re.p, 0, sizeof(int32_t) * (2 * (size_t)m + 1), s));
        hipLaunchKernelGGL(k_band_collect, dim3((unsigned)m * COLLECT_GROUPS), dim3(256), 0, s, f);
        // one-wavefront workgroups: as many as the LDS holds per CU, at most 16
        const int band_per_cu = std::min(16, std::max(1, (int)(163840 / (lds_band + sizeof(int) * (BT_MAX_SERIES + 1)))));
        hipLaunchKernelGGL(k_batch_band, dim3((unsigned)(num_cu * band_per_cu)), dim3(64), lds_band, s, f,
                           band_rows, maxT);
        hipLaunchKernelGGL(k_batch_final, dim3(m), dim3(FINAL_BLOCK), lds_f, s, f);
        if ((rc = check_launch("k_batch finalisation"))) return rc;
        ABC_HIP(hipMemcpyAsync(rech.data(), b_re.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
        ABC_HIP(hipMemcpyAsync(cnt.data(), out_count, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
        ABC_HIP(hipMemcpyAsync(used_h.data(), out_used, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
        ABC_HIP(hipStreamSynchronize(s));
        ++phases;
        for (int s2 = 0; s2 < m; ++s2) rechecked += rech[s2];
        bool overflow = false, short_q = false;
        for (int s2 = 0; s2 < m; ++s2) {
            overflow |= cnt[s2] < 0;
            short_q |= cnt[s2] >= 0 && cnt[s2] < quota && used_h[s2] < max_samples;
        }
        const bool stopped = stop_at >= 0 && rounds > stop_at;
        if (overflow || !short_q || !stopped || phases >= BT_MAX_PHASES) break;
        hipLaunchKernelGGL(k_batch_retarget, dim3((m + 255) / 256), dim3(256), 0, s, a, out_count, margin);
        if ((rc = check_launch("k_batch_retarget"))) return rc;
        phase0 = rounds;
        stop_at = -1;
    }
    hipLaunchKernelGGL(k_batch_moments, dim3(m), dim3(256), 0, s, out_theta, f.out_w, out_count,
                       quota, out_mean, out_cov);
    if ((rc = check_launch("k_batch moments"))) return rc;
    unsigned long long days = 0;
    ABC_HIP(hipMemcpyAsync(&days, b_days.p, sizeof(days), hipMemcpyDeviceToHost, s));
    ABC_HIP(hipStreamSynchronize(s));
    ABC_HIP(hipEventRecord(ev, s));
    ABC_HIP(hipStreamWaitEvent(user, ev, 0));
    if (stats) {
        stats->rounds = rounds;
        stats->graph_replays = polls;
        stats->sample_days = (int64_t)days;
        stats->rechecked = rechecked;
        stats->phases = phases;
        stats->grid = (int32_t)grid;
        stats->block = block;
        stats->spl = spl;
        stats->lds_bytes = (int32_t)(lds + static_lds);
        stats->rounds_ms = rounds_ms;
    }
    for (int s2 = 0; s2 < m; ++s2) {
        if (cnt[s2] < 0) {
            SeriesState st{};
            (void)hipMemcpy(&st, a.state + s2, sizeof(st), hipMemcpyDeviceToHost);
            return set_error(ABC_EOVERFLOW,
                             "series %d: %lld candidates exceed the capacity %d (float32 accepts %d of "
                             "target %d; folded: accepts %d, candidates %d, samples %lld of %lld; "
                             "%lld rounds, stop %lld)",
                             s2, (long long)-cnt[s2], cand_cap, st.acc, st.target, st.acc_f, st.cand_f,
                             (long long)st.done, (long long)st.next, (long long)rounds,
                             (long long)stop_at);
        }
        if (cnt[s2] < quota)
            return set_error(ABC_EOVERFLOW, "series %d: %lld of %d accepted within max_samples",
                             s2, (long long)cnt[s2], quota);
    }
    if (stop_at < 0 && (rounds == 0 || !flag_host[(rounds - 1) % BT_EVR]))
        return set_error(ABC_EOVERFLOW, "stopped after %lld rounds before every quota was met",
                         (long long)rounds);
    return ABC_OK;
}

extern "C" abc_status abc_set_batch_margin(int32_t margin)
{
    ABC_REQUIRE(margin >= -(1 << 20) && margin <= (1 << 20), "margin must be within +-2^20");
    g_batch_margin = margin;
    return ABC_OK;
}

extern "C" abc_status abc_batch_run(const abc_batch_series* series, int32_t m,
                                    const abc_prior* prior, const abc_model* model,
                                    uint64_t seed, uint32_t domain, int32_t quota,
                                    int64_t round_size, int64_t max_samples, float band_w,
                                    int32_t rounds_per_graph, int32_t cand_capacity,
                                    int64_t* out_idx,
                                    float* out_theta, float* out_dist, int64_t* out_count,
                                    int64_t* out_used, double* out_mean, double* out_cov,
                                    abc_batch_stats* stats, void* stream)
{
    return batch_run(series, m, prior, model, seed, domain, quota, round_size, max_samples, band_w,
                     rounds_per_graph, cand_capacity, nullptr, out_idx, out_theta, nullptr, out_dist,
                     out_count, out_used, out_mean, out_cov, stats, stream);
}

extern "C" abc_status abc_batch_run_weighted(const abc_batch_series* series, int32_t m,
                                             const abc_prior* prior, const abc_model* model,
                                             uint64_t seed, uint32_t domain, int32_t quota,
                                             int64_t round_size, int64_t max_samples, float band_w,
                                             int32_t rounds_per_graph, int32_t cand_capacity,
                                             const abc_batch_proposal* prop, int64_t* out_idx,
                                             float* out_theta, float* out_w, float* out_dist,
                                             int64_t* out_count, int64_t* out_used, double* out_mean,
                                             double* out_cov, abc_batch_stats* stats, void* stream)
{
    ABC_REQUIRE(prop != nullptr, "proposal is NULL");
    return batch_run(series, m, prior, model, seed, domain, quota, round_size, max_samples, band_w,
                     rounds_per_graph, cand_capacity, prop, out_idx, out_theta, out_w, out_dist,
                     out_count, out_used, out_mean, out_cov, stats, stream);
}
