/*
 * abc.h -- C ABI of libabc.so, the MI355X (gfx950) rejection-ABC hot path for
 * the stochastic COVID-19 compartment model of Kulkarni, Krell, Nabarro and
 * Moritz, "Hardware-accelerated Simulation-based Inference of Stochastic
 * Epidemiology Models for COVID-19" (arXiv 2012.14332).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named "device" are HIP device memory owned by the caller; host
 *    structs are read during the call only. The library keeps no caller
 *    pointer after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Every
 *    call only enqueues work on it and returns; results are visible after the
 *    stream has been synchronised.
 *  - Return value: ABC_OK, or a negative status. Argument errors are detected
 *    on the host before anything is enqueued (ABC_EINVAL); HIP failures
 *    return ABC_EHIP. abc_last_error() gives a message for the calling thread.
 *  - Results are a pure function of the arguments: the seed, stream domain,
 *    series id and sample indices fix every random number (counter-based
 *    Philox4x32-10), so launch shapes and call splitting never change them.
 *
 * Parameter vector (eq. 1): theta = [alpha0, alpha, n, beta, gamma, delta,
 * eta, kappa], stored as 8 consecutive float32 per sample ([n][8] row-major).
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = (seed mod
 * 2^32, seed >> 32) and counter = (i mod 2^32, i >> 32, series,
 * (day << 8) | (domain << 4) | block) for sample index i.
 *   theta draw (eq. 2): day 0, blocks 0..1 -> 8 words w; u = (w >> 8) 2^-24;
 *     theta_k = fmaf(hi_k - lo_k, u_k, lo_k) in float32.
 *   noise of day t >= 1: block 0 -> four words -> six 21-bit fields
 *     (w0..w3 >> 11, (w0 & 0x7ff) << 10 | (w1 & 0x3ff),
 *     (w2 & 0x7ff) << 10 | (w3 & 0x3ff)); u = (f + 1/2) 2^-21; Box-Muller
 *     pairs (u0,u1), (u2,u3), (u4,u5) give z1..z5, one per transition.
 */
#ifndef ABC_H
#define ABC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define ABC_API __attribute__((visibility("default")))
#else
#define ABC_API
#endif

typedef int32_t abc_status;
#define ABC_OK 0
#define ABC_EINVAL (-1)       /* bad argument; nothing enqueued */
#define ABC_EHIP (-2)         /* a HIP runtime call failed */
#define ABC_ENOMEM (-3)       /* library scratch could not be allocated */
#define ABC_EUNSUPPORTED (-4) /* option combination not built */
#define ABC_EOVERFLOW (-5)    /* a result did not fit its buffer, or a quota was not met */

/* Model options (flags of abc_model.flags). */
#define ABC_FP64 0x1u          /* simulate in double precision (default float32) */
#define ABC_KAHAN 0x2u         /* compensated float32 distance sum */
#define ABC_NOISE_LITERAL 0x4u /* noise sd = h^(1/4) ("variance sqrt(h)" read literally);
                                  default sd = sqrt(h), i.e. variance h */
#define ABC_DIST_RAW 0x8u      /* Euclidean distance on raw counts (default: log1p counts) */
#define ABC_SUPPORT 0x10u      /* supplied theta: rows outside the closed prior box have prior
                                  density zero and get distance +INF without simulation */
#define ABC_NO_BOUND 0x20u     /* float32 early exit on the running sum alone: no lower bound
                                  on the days still to come from the cumulative R and D */

#define ABC_T_MAX 1024         /* longest horizon a series may have */

/* Uniform prior box (eq. 2): theta_k ~ U(lo_k, hi_k), lo_k <= hi_k. The paper's
 * prior is lo = 0, hi = [1, 100, 2, 1, 1, 1, 1, 2]. Host memory. */
typedef struct {
    float lo[8];
    float hi[8];
} abc_prior;

/* Random stream selector. domain in [0, 15]: 0 = observation synthesis,
 * 1 = ABC sampling/simulation, 2 = learned-proposal training data,
 * 3 = network initialisation, 5 = learned-proposal draws, 6 = projections,
 * 7 = ABC-SMC generations >= 1. */
typedef struct {
    uint64_t seed;
    uint32_t domain;
    uint32_t series;
} abc_stream;

/* One observed series (Sec. 2.1): population P at the first time point,
 * observed A0, R0, D0 at day 0, horizon T in [1, ABC_T_MAX], and the observed
 * A, R, D counts of days 1..T as a DEVICE int32 array [3][T] (row c = A, R, D).
 * obs may be NULL for calls that do not compare (abc_simulate_record).
 * Requires A0 >= 1, R0, D0 >= 0 and A0 + R0 + D0 <= P <= 2^31 - 1 (the state is
 * int32). I0 = floor(kappa A0) is limited to P - A0 - R0 - D0 so that S >= 0. */
typedef struct {
    int64_t P;
    int32_t A0, R0, D0;
    int32_t T;
    const int32_t* obs;
} abc_series;

/* Model options: noise_scale multiplies the noise standard deviation
 * (1 = the paper's model, 0 = the deterministic floor map); flags = ABC_*. */
typedef struct {
    float noise_scale;
    uint32_t flags;
} abc_model;

/*
 * Draw theta for samples first .. first+n-1 from the uniform prior (eq. 2).
 *   prior   host; lo <= hi elementwise (finite).
 *   st      host; stream selector (domain <= 15).
 *   theta   device float32 [n][8], written.
 * n = 0 is a no-op. Errors: ABC_EINVAL (NULL pointer, bad box, n < 0).
 */
ABC_API abc_status abc_sample_prior(const abc_prior* prior, const abc_stream* st, uint64_t first,
                            int64_t n, float* theta, void* stream);

/*
 * Simulate the tau-leap model of Sec. 2.1 (eqs. 3-5: hazards, Gaussian draws
 * floored and clamped in h order, day updates) for samples first .. first+n-1
 * and reduce each trajectory to its Euclidean distance from ser->obs over days
 * 1..T (Sec. 2.2), on log1p counts unless ABC_DIST_RAW.
 *   ser     host struct; ser->obs device [3][T] (required).
 *   model   host; noise scale and ABC_* flags.
 *   st      host; stream selector.
 *   theta   device float32 [n][8] with non-negative rates, or NULL: then theta
 *           is drawn in-kernel from `prior` (lo >= 0) on the same stream exactly
 *           as abc_sample_prior would.
 *   prior   host; required when theta is NULL or the ABC_SUPPORT flag is set,
 *           ignored otherwise. With ABC_SUPPORT and supplied theta, a row with
 *           any theta_k < lo_k, theta_k > hi_k (or NaN) is not simulated and
 *           reports dist +INF.
 *   eps_exit  early-exit bound: a sample stops as soon as its running squared
 *           distance exceeds eps_exit^2 (with a margin that can never flip an
 *           accept decision at eps <= eps_exit) and reports +INF. For the
 *           float32 log1p distance the running sum is first raised by a lower
 *           bound on the days still to come (recovered and dead counts never
 *           fall, so a count already above a later observation must still pay
 *           for it), kept below what float32 rounding could undo; ABC_NO_BOUND
 *           turns that off. Either way +INF means the float32 distance would
 *           have ended above eps_exit. Pass +INF to simulate every day.
 *   dist    device float32 [n]: the distance, or +INF after an early exit.
 *   dist64  device float64 [n] or NULL: the same value before rounding to
 *           float32 (with ABC_FP64 the full double result).
 *   days    device uint64 or NULL: the float32 kernel adds the number of
 *           sample-days it simulated (after early exits) to *days.
 * Errors: ABC_EINVAL (T out of range, P/A0/R0/D0 inconsistent, NULL pointers,
 * n < 0, noise_scale < 0 or not finite).
 */
ABC_API abc_status abc_simulate_distance(const abc_series* ser, const abc_model* model,
                                 const abc_stream* st, const float* theta,
                                 const abc_prior* prior, uint64_t first, int64_t n,
                                 float eps_exit, float* dist, double* dist64,
                                 unsigned long long* days, void* stream);

/*
 * Several series in one persistent launch (Sec. 3.1: many independent
 * samples in parallel; here the samples of up to ABC_MULTI_MAX series share
 * one launch instead of one launch per series). Job j simulates samples
 * first .. first+n-1 of series `ser` on stream (seed, domain, series) with
 * theta drawn in-kernel from `prior` (as abc_simulate_distance with theta =
 * NULL), early exit at eps_exit, and writes dist [n] -- bit for bit what
 * abc_simulate_distance would write for that job. The 64-sample chunks of
 * all jobs form one queue, longest horizon first, so the launch ends with one
 * tail of short trajectories instead of one per series.
 *   jobs    host array [m], 1 <= m <= ABC_MULTI_MAX; each ser->obs device [3][T];
 *           dist device float32 [n] (NULL allowed when n = 0).
 *   model   float32 path only: ABC_FP64 and ABC_SUPPORT are rejected.
 *   days    device uint64 or NULL: += sample-days simulated over all jobs.
 * The observed rows and the future-days bound tables of all jobs live in the
 * workgroup's LDS; tables get coarser time blocks (a weaker bound, never a
 * different distance) when they would not fit, and the launch shape set by
 * abc_set_launch_config gives the workgroup size and at most blocks_per_cu
 * resident workgroups per CU (fewer when the LDS allows fewer).
 * Errors: ABC_EINVAL (m out of range, a job's series, n or eps_exit invalid,
 * total n > 2^36, unsupported flags), ABC_EUNSUPPORTED (the observed rows
 * alone exceed the LDS of a workgroup).
 */
#define ABC_MULTI_MAX 8
typedef struct {
    const abc_series* ser;  /* host struct; ser->obs device [3][T] */
    uint32_t series;        /* stream series id of the job */
    uint32_t pad;
    uint64_t first;         /* first sample index */
    int64_t n;              /* samples */
    float eps_exit;         /* early-exit bound (+INF: none) */
    uint32_t pad2;
    float* dist;            /* device float32 [n] */
} abc_sim_job;
ABC_API abc_status abc_simulate_distance_multi(const abc_sim_job* jobs, int32_t m,
                                       const abc_model* model, const abc_prior* prior,
                                       uint64_t seed, uint32_t domain,
                                       unsigned long long* days, void* stream);

/*
 * Simulate like abc_simulate_distance but record the full integer state
 * (S, I, A, R, D, Ru) of days 0..T: traj is device int32 [n][T+1][6].
 * ser->obs is not read. theta is device float32 [n][8] (required).
 * Used to synthesise observed series (domain 0) and to check trajectories.
 */
ABC_API abc_status abc_simulate_record(const abc_series* ser, const abc_model* model,
                               const abc_stream* st, const float* theta, uint64_t first,
                               int64_t n, int32_t* traj, void* stream);

/*
 * Float64 decision for borderline samples of a float32 pass. The float32
 * distance of a trajectory can differ from its float64 value by more than a
 * few ulps once a rounding moves a floored count (Sec. 2.1 draws); this call
 * makes the accept decision (dist <= eps, eq. 7) in float64 wherever the
 * float32 distance falls inside the band (eps (1 - band_w), eps (1 + band_w)].
 * Input: the candidate rows of abc_accept_compact run with eps (1 + band_w)
 * (idx, theta, dist, optional weight, all device, `capacity` rows) and their
 * device count. Each in-band row is simulated again in float64 (same stream,
 * sample idx[r], theta[r]) and its dist replaced by the float64 distance
 * rounded to float32; rows outside the band keep their float32 decision.
 * Kept rows are compacted in place in their original order and *count is set
 * to their number. If *count > capacity on entry (an overflowed candidate
 * set) nothing is changed. rechecked (device int32, nullable) receives the
 * number of rows simulated in float64. ser, model, st as for
 * abc_simulate_distance (the ABC_FP64 and ABC_KAHAN flags are ignored).
 * eps = +INF keeps every row (nothing lies inside an infinite band); at
 * eps = 0 the band has no width, so an exact-match decision needs rows from
 * an ABC_FP64 pass. Errors: ABC_EINVAL (eps < 0 or NaN, band_w outside [0, 1),
 * NULL pointers, T too long for the float64 row kernel's LDS).
 */
ABC_API abc_status abc_recheck_band(const abc_series* ser, const abc_model* model,
                                    const abc_stream* st, float eps, float band_w,
                                    int64_t capacity, int64_t* idx, float* theta, float* dist,
                                    float* weight, int64_t* count, int32_t* rechecked,
                                    void* stream);

/*
 * Accept-reject and stable compaction (Sec. 2.2, eq. 7; Sec. 3.2): keep the
 * samples k in [0, n) with dist[k] <= eps, in increasing k, and write for the
 * r-th kept sample (r < capacity):
 *   out_idx[r]   = first + k                          (device int64 [capacity])
 *   out_theta[r] = theta[k][0..7]                     (device float32 [capacity][8])
 *   out_dist[r]  = dist[k]                            (device float32 [capacity], nullable)
 *   out_w[r]     = weight[k]                          (device float32 [capacity], nullable)
 * theta may be NULL: then the row is re-drawn from `prior` on stream `st`
 * (the in-kernel draw of abc_simulate_distance). weight may be NULL (then
 * out_w must be NULL). *out_count (device int64) receives the total number
 * kept, which may exceed capacity; rows beyond capacity are not written.
 * Errors: ABC_EINVAL (NULL required pointer, n < 0, capacity < 0, theta and
 * prior both NULL).
 */
ABC_API abc_status abc_accept_compact(const float* dist, const float* theta, const float* weight,
                              const abc_prior* prior, const abc_stream* st, int64_t n,
                              uint64_t first, float eps, int64_t capacity, int64_t* out_idx,
                              float* out_theta, float* out_dist, float* out_w,
                              int64_t* out_count, void* stream);

/*
 * abc_accept_compact for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments, layout, result and errors; the caller still
 * passes every input and output. The compaction's scratch (one status word
 * per tile of 16384 or 65536 samples, plus a ticket) lives in a fixed
 * library-owned device array of about 128 KiB, which each GPU the library runs
 * on holds until the process ends; the call makes no hipMalloc, hipFree or
 * other allocating call, and clears the scratch with a kernel, not a memset.
 * n is limited to ABC_NOALLOC_COMPACT_MAX_N (larger n: ABC_EINVAL). Every call
 * on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or host threads) race and must be serialised by the
 * caller; calls in one stream are ordered and safe.
 */
#define ABC_NOALLOC_COMPACT_MAX_N ((int64_t)1 << 30)
ABC_API abc_status abc_accept_compact_noalloc(const float* dist, const float* theta,
                                      const float* weight, const abc_prior* prior,
                                      const abc_stream* st, int64_t n, uint64_t first, float eps,
                                      int64_t capacity, int64_t* out_idx, float* out_theta,
                                      float* out_dist, float* out_w, int64_t* out_count,
                                      void* stream);

/*
 * Posterior mean and covariance of accepted theta in float64 (the summaries
 * the paper reports as posterior averages, Table "t:trajectories").
 *   theta   device float32 [n_max][8], 16-byte aligned; the first n rows are
 *           used, where n = min(*n_dev, n_max) is read on the device (n_dev:
 *           device int64, e.g. the out_count of abc_accept_compact). n_dev may
 *           be NULL: n = n_max.
 *   weight  device float32 [n_max] or NULL (all ones).
 *   mean    device float64 [8]: sum w theta / V1.
 *   cov     device float64 [8][8]: sum w (theta-mean)(theta-mean)^T / (V1 - V2/V1),
 *           V1 = sum w, V2 = sum w^2 (the unbiased n-1 form when w = 1).
 * n = 0 gives NaN mean and covariance; n = 1 a NaN covariance. The summation
 * order depends only on n (fixed contiguous row ranges), never on timing or
 * on the device. Errors: ABC_EINVAL (n_max < 0, NULL or misaligned theta,
 * NULL mean/cov).
 */
ABC_API abc_status abc_posterior_moments(const float* theta, const float* weight, const int64_t* n_dev,
                                 int64_t n_max, double* mean, double* cov, void* stream);

/*
 * Launch shape of the float32 simulate+distance kernel for later calls made
 * by the calling thread (the autotuner's knob): spl = independent samples
 * per lane (1, 2, 4 or 8; more than 1 only for the default noise and
 * distance), block = workgroup size (multiple of 64 in [64, 1024/spl]),
 * blocks_per_cu = resident workgroups per compute unit (1..64). A 0 selects
 * that argument's default: spl 1, block 512 / spl (at least 64), blocks_per_cu
 * 2 (two 512-thread workgroups per CU were the fastest plain three-country
 * step on MI355X). Results
 * never depend on these settings, only speed.
 */
ABC_API abc_status abc_set_launch_config(int32_t spl, int32_t block, int32_t blocks_per_cu);
ABC_API abc_status abc_get_launch_config(int32_t* spl, int32_t* block, int32_t* blocks_per_cu);

/* Lane-refill threshold of the float32 refill kernels (abc_simulate_distance
 * and abc_batch_run) for the calling thread: a wavefront refills its idle
 * lanes from its queue once at least `lanes` of its 64 lanes are idle
 * (1 = at every step; default 8). Results never depend on it.
 * Errors: ABC_EINVAL unless 1 <= lanes <= 64 (0 selects the default). */
ABC_API abc_status abc_set_refill_min(int32_t lanes);
ABC_API int32_t abc_get_refill_min(void);

/* Margin of abc_batch_run's first target for the calling thread: every series
 * takes samples until its float32 accepts reach quota + margin (at least 1),
 * then the run is finalised; a series left with fewer than quota rows after
 * the float64 band decision continues its stream (see abc_batch_run).
 * 0 selects the default max(4, quota / 256). A negative margin makes the
 * first finalisation come early, so that the continuation runs; results
 * never depend on it. Errors: ABC_EINVAL unless |margin| <= 2^20. */
ABC_API abc_status abc_set_batch_margin(int32_t margin);

/* One observed series of a batch: as abc_series, plus its tolerance and its
 * stream series id (counter word 2; give every series of a batch its own). */
typedef struct {
    int64_t P;
    int32_t A0, R0, D0;
    int32_t T;
    const int32_t* obs;  /* device [3][T] */
    float eps;
    uint32_t series;
} abc_batch_series;

typedef struct {
    int64_t rounds;        /* rounds run */
    int64_t graph_replays; /* completion flags the host read */
    int64_t sample_days;   /* sample-days simulated (after early exits) */
    int64_t rechecked;     /* candidates decided in float64 */
    int32_t grid, block, spl, lds_bytes;
    float rounds_ms;       /* wall time of the rounds (host waits included) */
    int32_t phases;        /* finalisations run (more than 1 when one kept fewer than quota rows) */
} abc_batch_stats;

/*
 * Rejection ABC over m observed series of uneven T and P in one persistent
 * launch per round (Sec. 3.1: repeat until the target number of accepted
 * samples; Sec. 3.2: accept-reject on the device), until every series has
 * `quota` accepted samples. Each round hands round_size samples, split evenly,
 * to the series still short of their target; series j consumes its stream indices
 * 0, 1, 2, ... as a prefix (theta drawn from `prior` on stream (seed, domain,
 * series[j].series)). Each round is planned on the device from the counts of
 * the rounds up to two before it, so consecutive rounds overlap (they
 * alternate between two streams of the call); a completion flag follows
 * every round and the host reads the flag of the round rounds_per_graph
 * (clamped to [2, 6]) rounds back. Which samples are simulated, and so every
 * output, does not depend on that setting. At the end the candidates inside the
 * band (eps (1 - band_w), eps (1 + band_w)] are decided in float64, and the
 * first `quota` accepted samples by index are written per series:
 *   out_idx   device int64 [m][quota]        out_theta device float32 [m][quota][8]
 *   out_dist  device float32 [m][quota]      out_count device int64 [m] (rows written)
 *   out_used  device int64 [m] (samples simulated per series)
 *   out_mean  device float64 [m][8]          out_cov   device float64 [m][8][8]
 * The result equals the first `quota` indices i with dist_i <= eps of the
 * plain path. Only the default model (flags = 0, any noise_scale) runs here.
 * m <= 256; quota <= 4096; the series descriptors (64 B each) and the launch
 * shape's ring must fit in LDS (the observed series are read from device
 * memory), otherwise ABC_EUNSUPPORTED. max_samples bounds the
 * samples per series; ABC_EOVERFLOW if some series then still lacks its quota
 * or produced more candidates (d <= eps (1 + band_w)) than cand_capacity rows
 * (0 = max(4 quota, 256), at most 16384, and the finalisation sorts them in LDS: about
 * 12 B per row must fit, so 8192 rows at most on gfx950). Each round caps a series' share so
 * that the running round's and its own expected candidates stay within half the free capacity,
 * at an upper bound of the candidate rate so far ((sqrt(c + 1) + 2)^2 candidates for c counted),
 * and to the samples its target still needs at a lower bound of its accept rate. A series'
 * target counts float32 accepts (d <= eps (1 - 1e-5)), first quota + max(4, quota / 256); when the
 * finalisation keeps fewer than quota rows of a series (float64 decisions moved accepts
 * across eps), its target rises by the shortfall and the margin and the rounds continue
 * its stream before a further finalisation (at most 8 in all; stats->phases counts them).
 * Launch shape: abc_set_launch_config (spl 1, 2, 4 or 8). Blocks the calling host thread until
 * done; the caller's stream is ordered before and after the work. stats may be NULL.
 */
ABC_API abc_status abc_batch_run(const abc_batch_series* series, int32_t m,
                                 const abc_prior* prior, const abc_model* model, uint64_t seed,
                                 uint32_t domain, int32_t quota, int64_t round_size,
                                 int64_t max_samples, float band_w, int32_t rounds_per_graph,
                                 int32_t cand_capacity, int64_t* out_idx, float* out_theta,
                                 float* out_dist,
                                 int64_t* out_count, int64_t* out_used, double* out_mean,
                                 double* out_cov, abc_batch_stats* stats, void* stream);

/* Learned proposal of a batched run (not in the paper): per series a row of
 * the network output (abc_mdn_forward of the series' features), drawn as the
 * defensive mixture of abc_mdn_sample with the prior box `prior`. */
typedef struct {
    const float* mix;   /* device float32 [m][136], row s for series s */
    float lambda;       /* defensive prior weight in [0, 1] */
    float inflate;      /* factor on every component sd, [1, 100] */
    uint32_t domain;    /* stream domain of the proposal draws (5 in this build) */
    uint32_t pad;
} abc_batch_proposal;

/*
 * abc_batch_run with theta drawn from the learned proposal instead of the
 * prior: sample i of series s takes theta and its importance weight
 * prior/proposal from abc_mdn_sample's draw on stream (seed, prop->domain,
 * series id, i), and its simulation noise from (seed, domain, series id, i)
 * as in abc_batch_run. Outputs as abc_batch_run plus out_w (device float32
 * [m][quota]); out_mean / out_cov are the weighted moments (sum w theta / V1,
 * sum w (theta - mean)(theta - mean)^T / (V1 - V2/V1)). The kept rows are the
 * first `quota` accepted by index, so the result equals the per-series
 * learned-proposal pass run until the same quota. Errors as abc_batch_run,
 * plus ABC_EINVAL for a NULL proposal or out_w, lambda outside [0, 1],
 * inflate outside [1, 100], or prop->domain equal to `domain` (theta's words
 * would then be the simulation's day-1 noise words).
 */
ABC_API abc_status abc_batch_run_weighted(const abc_batch_series* series, int32_t m,
                                          const abc_prior* prior, const abc_model* model,
                                          uint64_t seed, uint32_t domain, int32_t quota,
                                          int64_t round_size, int64_t max_samples, float band_w,
                                          int32_t rounds_per_graph, int32_t cand_capacity,
                                          const abc_batch_proposal* prop, int64_t* out_idx,
                                          float* out_theta, float* out_w, float* out_dist,
                                          int64_t* out_count, int64_t* out_used, double* out_mean,
                                          double* out_cov, abc_batch_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Learned proposal (not in the paper, whose proposal is the prior): a
 * mixture-density network q(theta | x) trained on (theta, x) pairs that the
 * simulator itself produces, used as an importance-sampling proposal for
 * rejection ABC at the same eps. x = log1p(A, R, D) at 32 evenly spaced days
 * d_k = 1 + rint(k (T - 1) / 31), k = 0..31 (96 float32, A block first),
 * standardised per feature; theta standardised by the prior's mean and sd.
 * Network 96 -> 256 -> 256 -> 136 (exact-erf GELU), output = 8 logits,
 * 8x8 means, 8x8 log sd (clamped to [-7, 3]) of a diagonal Gaussian mixture.
 * Products in bfloat16 on MFMA with float32 accumulation; parameters, loss,
 * gradients and Adam in float32. The handle owns all device memory.
 * ------------------------------------------------------------------------ */
typedef struct abc_mdn abc_mdn;

/* Number of float32 parameters: W1 [96][256], b1 [256], W2 [256][256], b2,
 * W3 [256][136], b3 [136], in this order, W stored [fan_in][fan_out]. */
ABC_API int64_t abc_mdn_param_count(void);

/* Create a network for the prior box `prior` (host) with weights drawn
 * U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from stream (init_seed, domain 3),
 * biases 0, feature standardisation mean 0 / sd 1. Synchronises the device. */
ABC_API abc_status abc_mdn_create(const abc_prior* prior, uint64_t init_seed, abc_mdn** out);
ABC_API abc_status abc_mdn_destroy(abc_mdn* net);

/* Device pointers (owned by the net) to the float32 parameters and to the
 * gradient of the last abc_mdn_loss_grad / training step, both
 * [abc_mdn_param_count()]. After writing parameters, call abc_mdn_sync_params. */
ABC_API abc_status abc_mdn_params(abc_mdn* net, float** params, float** grads);
ABC_API abc_status abc_mdn_sync_params(abc_mdn* net, void* stream);
/* Copy the float32 parameters in from / out to a device buffer
 * [param_count] (set also refreshes the bfloat16 copies). */
ABC_API abc_status abc_mdn_set_params(abc_mdn* net, const float* src, void* stream);
ABC_API abc_status abc_mdn_get_params(const abc_mdn* net, float* dst, void* stream);
/* Copy out the feature standardisation (device float32 [96] each). */
ABC_API abc_status abc_mdn_get_standardizer(const abc_mdn* net, float* mean96, float* sd96,
                                            void* stream);

/* Training pairs: for samples first..first+n-1 of stream (seed, domain,
 * series): theta from `prior` (blocks 0-1 of day 0, as abc_sample_prior);
 * T = T_lo + floor(u (T_hi - T_lo + 1)) and P = rint(10^(log10P_lo + u'
 * (log10P_hi - log10P_lo))) from block 2 of day 0 (u, u' from its first two
 * words as in the theta draw); A0 active at day 0, R0 = D0 = 0; the float32
 * model of abc_simulate_distance on the same stream; features as above,
 * unstandardised. Outputs device: features [n][96], theta [n][8], TP [n][2]
 * (T, P; nullable). */
ABC_API abc_status abc_mdn_simulate_features(const abc_prior* prior, uint64_t seed,
                                             uint32_t domain, uint32_t series, uint64_t first,
                                             int64_t n, int32_t T_lo, int32_t T_hi,
                                             double log10P_lo, double log10P_hi, int32_t A0,
                                             float* features, float* theta, int32_t* TP,
                                             void* stream);

/* The 96 unstandardised features of an observed series (ser->obs device). */
ABC_API abc_status abc_series_features(const abc_series* ser, float* out96, void* stream);

/* Per-feature mean and sd (float64 two-pass, sd floored at 1e-6) of
 * features [n][96] (device), kept in the net for every later call. */
ABC_API abc_status abc_mdn_fit_standardizer(abc_mdn* net, const float* features, int64_t n,
                                            void* stream);

/* Network outputs [n][136] (device, float32) for unstandardised features [n][96].
 * Every entry point below that takes features [n][96] requires them 16-byte
 * aligned (ABC_EINVAL otherwise): the first layer reads them four at a time. */
ABC_API abc_status abc_mdn_forward(abc_mdn* net, const float* features, int64_t n, float* out,
                                   void* stream);

/* Mean negative log-likelihood of theta [n][8] (original units) under the
 * network's mixture for features [n][96], and its gradient w.r.t. the float32
 * parameters (device float32 loss scalar and grad [param_count], nullable). */
ABC_API abc_status abc_mdn_loss_grad(abc_mdn* net, const float* features, const float* theta,
                                     int64_t n, float* loss, float* grad, void* stream);

/* Adam (beta 0.9, 0.999, eps 1e-8, learning rate lr) on the mean NLL over
 * `epochs` passes of n pairs in batches of `batch` (floor(n / batch) steps per
 * epoch; epoch e visits row (a_e j + c_e) mod n, with (a_e, c_e) from
 * shuffle_seed). One training step is captured once as a hipGraph and
 * replayed. loss_log (device float32 [steps], nullable) receives each step's
 * batch loss; steps_out and train_ms (host, nullable) the step count and the
 * GPU time of the replays. Blocks the host until done. */
ABC_API abc_status abc_mdn_train(abc_mdn* net, const float* features, const float* theta,
                                 int64_t n, int32_t epochs, int32_t batch, float lr,
                                 uint64_t shuffle_seed, float* loss_log, int64_t* steps_out,
                                 float* train_ms, void* stream);

/* Proposal draws for samples first..first+n-1 of stream st: with probability
 * lambda theta ~ prior, otherwise from the mixture given by `mix` (device,
 * one network output row [136]) with every component sd multiplied by
 * `inflate` (>= 1; the network estimates the eps -> 0 posterior, which is
 * narrower than the eps-ABC posterior) and every component truncated to the
 * prior box dimension by dimension (inverse-CDF draws, one per dimension; a
 * component whose mass in the box is below 1e-30 in some dimension is
 * dropped). Day 1 of the stream: block 0 words 0, 1 choose prior/mixture and
 * the component, blocks 1-2 give the eight uniforms. weight = prior(theta) /
 * q(theta), q = (1 - lambda) q_trunc + lambda prior, q_trunc the truncated
 * mixture's density. Outputs device theta [n][8], weight [n]. The caller
 * simulates these samples on another domain than st->domain: day 1 of
 * st->domain supplies theta here, and the same words as simulation noise would
 * tie each sample to its own trajectory. */
ABC_API abc_status abc_mdn_sample(const abc_mdn* net, const float* mix, float lambda,
                                  float inflate, const abc_stream* st, uint64_t first, int64_t n,
                                  float* theta, float* weight, void* stream);

/*
 * Posterior-predictive bands (Sec. 5: projections from accepted samples with
 * the 5th-95th percentile band): for every day 0..T and compartment
 * (S, I, A, R, D, Ru) the quantiles q[0..nq-1] (host, in [0, 1], nq <= 16) of
 * n <= 8192 recorded trajectories traj (device int32 [n][T+1][6], e.g. from
 * abc_simulate_record of accepted theta over a longer horizon). Quantile q
 * interpolates linearly between the order statistics at h = (n - 1) q.
 * out: device float32 [nq][T+1][6].
 */
ABC_API abc_status abc_trajectory_bands(const int32_t* traj, int64_t n, int32_t T,
                                        const double* q, int32_t nq, float* out, void* stream);

/*
 * Nearest-k rule (the "keep the k nearest prior samples" form of rejection
 * ABC, Sec. 2.2; the per-run Top-k return of Sec. 3.2): the k samples of a
 * launch with the smallest distances, ties to the lower sample index, in
 * sample-index order.
 *   dist    device float32 [n] (sample first + j at position j), n < 2^32.
 *   theta   device float32 [n][8] or NULL: then output rows are re-drawn from
 *           `prior` on stream `st` (as abc_accept_compact does).
 *   k       1 <= k <= min(n, 4096).
 *   out_idx device int64 [k]; out_theta device float32 [k][8] or NULL;
 *   out_dist device float32 [k] or NULL; out_kth device float32 [1] or NULL:
 *           the k-th smallest distance.
 * Exact selection by narrowing histograms (no full sort); synchronises the
 * stream once per narrowing pass (at most 7). NaN sorts above +inf.
 * Errors: ABC_EINVAL (bad sizes, NULL pointers, fewer than k finite
 * distances).
 */
ABC_API abc_status abc_nearest_k(const float* dist, const float* theta, const abc_prior* prior,
                                 const abc_stream* st, int64_t n, uint64_t first, int32_t k,
                                 int64_t* out_idx, float* out_theta, float* out_dist,
                                 float* out_kth, void* stream);

/*
 * Nearest-k among n <= 65536 rows with float64 distances (e.g. the float64
 * re-decision of the candidates of abc_nearest_k): the k rows with the
 * smallest (dist64, idx), written in increasing idx order. All pointers
 * device; theta / out_theta optional together; out_dist optional.
 * Errors: ABC_EINVAL.
 */
ABC_API abc_status abc_nearest_k_rows(const double* dist64, const int64_t* idx, const float* theta,
                                      int64_t n, int32_t k, int64_t* out_idx, float* out_theta,
                                      double* out_dist, void* stream);

/*
 * Float64 distances (Sec. 2.2) of listed rows: row q is sample idx[q] of
 * stream `st` with parameters theta[q] (device float32 [n][8]); the same
 * float64 simulation as abc_simulate_distance with ABC_FP64, without early
 * exit. dist64: device float64 [n]. ABC_SUPPORT is ignored.
 * Errors: ABC_EINVAL (NULL pointers, n < 0, series/model checks).
 */
ABC_API abc_status abc_simulate_rows_f64(const abc_series* ser, const abc_model* model,
                                         const abc_stream* st, const int64_t* idx,
                                         const float* theta, int64_t n, double* dist64,
                                         void* stream);

/*
 * ABC-SMC (Sec. 2.2 names sequential Monte Carlo ABC: a population refined
 * over a decreasing tolerance sequence). Population Monte Carlo ABC
 * (Beaumont, Cornuet, Marin & Robert 2009) with adaptive tolerances:
 *   generation 0: rejection ABC from `prior` at eps0 on stream (seed, domain 1,
 *     series); the population is the first N accepted samples by index, with
 *     equal weights.
 *   generation t >= 1: eps_t = max(eps_min, the ceil(alpha N)-th smallest
 *     float64 distance of generation t-1) rounded to float32; Sigma = 2 x the
 *     weighted covariance of generation t-1 (sums over particles left to
 *     right), L its Cholesky factor. Candidate i (stream domain 7, series word
 *     series | t << 16, day 0 blocks 0..2) draws a 53-bit uniform u and eight
 *     Box-Muller normals z; its ancestor is the smallest j with
 *     C_j > u C_{N-1} (C = running sums of the weights); theta* = theta_j + L z
 *     in float64, rounded to float32. Candidates outside the closed prior box
 *     are rejected without simulation; the others are simulated (days 1..T of
 *     the same stream) and accepted iff distance <= eps_t: with band_w > 0
 *     every candidate whose float32 distance is <= eps_t (1 + band_w) is
 *     decided by its float64 distance (which becomes the particle's distance);
 *     with band_w = 0 the float32 distance decides. The first N accepted
 *     by index form the population; weights W_i are proportional to
 *     1 / sum_j W_j exp(-(theta_i - theta_j)^T Sigma^-1 (theta_i - theta_j) / 2)
 *     (the uniform prior and the Gaussian normaliser cancel), normalised.
 * Every population is independent of chunk sizes and launch shapes.
 */
typedef struct {
    int32_t n_particles;  /* N in [2, 8192] (N >= 9 for a non-singular Sigma) */
    int32_t generations;  /* for abc_smc_run: at most this many, generation 0 included */
    double alpha;         /* (0, 1]: quantile of the next tolerance */
    float eps0;           /* tolerance of generation 0 */
    float eps_min;        /* floor of the tolerance sequence; abc_smc_run stops after the
                             generation that reaches it (0 = no floor) */
    float band_w;         /* [0, 1): candidates are float32 distances <= eps (1 + band_w),
                             decided in float64; 0 = float32 decisions */
    int32_t pad;
    int64_t chunk0;       /* candidates in the first chunk of a generation (doubling) */
    int64_t chunk_max;    /* largest chunk, <= 2^26 */
    int64_t max_samples;  /* candidate budget per generation: ABC_EOVERFLOW beyond it */
} abc_smc_config;

typedef struct {
    float eps;            /* tolerance of the generation */
    int32_t pad;
    int64_t samples;      /* candidates consumed: index of the N-th accepted + 1 */
    int64_t in_support;   /* of those, inside the prior box (= simulated) */
    int64_t proposed;     /* candidates drawn (whole chunks) */
    double ess;           /* 1 / sum W^2 */
} abc_smc_gen_stats;

/*
 * One generation `gen` of ABC-SMC for the observed series `ser` (float32 path;
 * ABC_FP64 is rejected). prev_theta [n_prev][8] float32, prev_w [n_prev]
 * (normalised) and prev_dist [n_prev] float64 are the previous generation
 * (device; ignored for gen 0). Outputs (device, cfg->n_particles rows):
 * idx (candidate index), theta (16-byte aligned), w (normalised float64
 * weights), dist (float64 distance of each particle, re-simulated in float64);
 * stats (host) as described above; ancestors (device int32 [N] or NULL):
 * index of each particle's ancestor in the previous population.
 * Workspace is allocated stream-ordered on `stream` and freed before return;
 * the call synchronises the stream once per chunk.
 * Errors: ABC_EINVAL (bad arguments, or a previous population whose Sigma is
 * not positive definite), ABC_EOVERFLOW (fewer than N accepted within
 * max_samples candidates), ABC_EHIP.
 */
ABC_API abc_status abc_smc_generation(const abc_series* ser, const abc_model* model,
                                      const abc_prior* prior, uint64_t seed, uint32_t series,
                                      int32_t gen, const float* prev_theta, const double* prev_w,
                                      const double* prev_dist, int32_t n_prev,
                                      const abc_smc_config* cfg, int64_t* idx, float* theta,
                                      double* w, double* dist, abc_smc_gen_stats* stats,
                                      int32_t* ancestors, void* stream);

/*
 * Generations 0, 1, ... of ABC-SMC (see abc_smc_generation) until
 * cfg->generations are done or a generation's tolerance reaches eps_min.
 * Outputs are device arrays with one block of N rows per generation:
 * idx [G][N], theta [G][N][8], w [G][N], dist [G][N]; stats host [G];
 * *gens_done (host) = generations completed. From generation 2 on, the first
 * chunk is sized from the previous generation's consumption (1.25 x its
 * samples, rounded up to chunk0 x 2^k, at most chunk_max); chunking never
 * changes a population.
 */
ABC_API abc_status abc_smc_run(const abc_series* ser, const abc_model* model,
                               const abc_prior* prior, uint64_t seed, uint32_t series,
                               const abc_smc_config* cfg, int64_t* idx, float* theta, double* w,
                               double* dist, abc_smc_gen_stats* stats, int32_t* gens_done,
                               void* stream);

/* Library scratch. Calls that need device scratch (compaction tiles, moment
 * partials, band flags, selection histograms, SMC work space, the batched
 * quota run's buffers) or a small pinned host buffer take it from
 * library-owned buffers kept per (device, stream): the first calls on a stream
 * allocate it (growing it synchronises that stream once), later calls reuse it
 * without allocating, so a steady-state call never waits for the device.
 * Calls on one stream are ordered and may share it; calls on one stream from
 * several host threads at once are not supported. abc_release_scratch()
 * synchronises the current device and frees every such buffer on it. */
ABC_API abc_status abc_release_scratch(void);

/* Message describing the last non-OK status returned on this thread. */
ABC_API const char* abc_last_error(void);

/* Library version string. */
ABC_API const char* abc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ABC_H */
