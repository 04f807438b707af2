// Host-side plumbing shared by the translation units of libabc.so: the
// per-thread error message, HIP error checks and argument validation.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/abc.h"

namespace abc {

abc_status set_error(abc_status st, const char* fmt, ...);

// LDS budget of a float64 row workgroup (several rows side by side per
// wavefront): small where the rows run beside a float32 launch, so that they
// do not crowd its workgroups out of the CU (the plain band decision), larger
// where they run alone (the SMC band decision, float64 row distances).
constexpr size_t ROW_LDS_BESIDE = 8192;
constexpr size_t ROW_LDS_ALONE = 20480;
// Float64 row wavefronts that spread rows over all SIMDs (one per SIMD) when
// the row kernel runs alone; beside a float32 launch the band decision
// spreads over up to twice as many.
constexpr int64_t ROW_WAVE_TARGET = 1024;

// Candidates a band-decision wavefront scans at least: beside a float32
// launch a few in-band rows (about a quarter of the candidates) share a
// wavefront; larger blocks (16, 32) slowed the float32 launches beside them
// (packed wavefronts live longer); alone the rows are spread for the
// shortest latency.
constexpr int32_t ROW_SCAN_BESIDE = 8;
constexpr int32_t ROW_SCAN_ALONE = 1;

// abc_recheck_band with a chosen LDS budget per row workgroup, grid cap and
// candidates per wavefront; with all_rows every candidate (not only those in
// the band) is decided by its float64 distance, and dist64 (nullable,
// [capacity]) receives that distance for each row, compacted with the rows.
abc_status recheck_band(const abc_series* ser, const abc_model* model, const abc_stream* st,
                        float eps, float band_w, int64_t capacity, int64_t* idx, float* theta,
                        float* dist, float* weight, int64_t* count, int32_t* rechecked,
                        void* stream, size_t lds_budget, int64_t grid_max, int32_t scan_min,
                        double* dist64, bool all_rows);

#define ABC_REQUIRE(cond, ...)                                 \
    do {                                                       \
        if (!(cond)) return ::abc::set_error(ABC_EINVAL, __VA_ARGS__); \
    } while (0)

#define ABC_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::abc::set_error(ABC_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

inline abc_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ABC_EHIP, "launch of %s: %s", what, hipGetErrorString(e));
    return ABC_OK;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Streaming loads of data read exactly once (distances, theta rows, weights):
// the non-temporal hint keeps them from displacing cached lines, worth about
// 6.9 instead of 6.1 TB/s on a plain read stream on MI355X.
typedef float abc_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float4* p)
{
    const abc_v4f t = __builtin_nontemporal_load(reinterpret_cast<const abc_v4f*>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ float load_stream(const float* p) { return __builtin_nontemporal_load(p); }

// Compute units and LDS bytes per workgroup of the current device, queried
// once per device (attribute queries cost tens of microseconds each, too much
// for a per-launch path).
struct DeviceInfo {
    int num_cu = 0;
    int max_lds = 0;
};
abc_status device_info(DeviceInfo* out);

// Library-owned scratch for the kernels a call enqueues on stream s: one
// device buffer per (device, stream, slot), grown to the largest request and
// kept (abc_release_scratch frees it). Consecutive calls on one stream reuse
// a slot's buffer, which stream order makes safe; growing it synchronises s
// once before the old buffer is freed. Unlike stream-ordered allocation, which
// on this runtime waits for the device, taking the buffer never blocks the
// host. Calls that enqueue their kernels and return use slot 0; a call that
// keeps its own scratch across nested calls on the same stream (the SMC
// generation around compaction and the band decision) uses higher slots.
constexpr int SCRATCH_LEAF = 0;
constexpr int SCRATCH_SMC_WS = 1;
constexpr int SCRATCH_SMC_SUMS = 2;
constexpr int SCRATCH_BATCH = 3;  // the batched quota run's buffers (its work runs on a stream of its own, ordered after and before s)
abc_status stream_scratch(hipStream_t s, size_t bytes, void** out, int slot = SCRATCH_LEAF);
// The same for pinned host memory (one buffer per (device, stream)), for
// small results a call reads back on the host.
abc_status stream_pinned(hipStream_t s, size_t bytes, void** out);

// Prior box -> (lo, width) with width = fl32(hi - lo), as the draw uses it.
inline abc_status prior_lo_width(const abc_prior* prior, float lo[8], float width[8])
{
    ABC_REQUIRE(prior != nullptr, "prior is NULL");
    for (int k = 0; k < 8; ++k) {
        ABC_REQUIRE(isfinite(prior->lo[k]) && isfinite(prior->hi[k]) && prior->lo[k] <= prior->hi[k],
                    "prior box %d is not finite with lo <= hi", k);
        lo[k] = prior->lo[k];
        width[k] = prior->hi[k] - prior->lo[k];
    }
    return ABC_OK;
}

inline abc_status check_stream_sel(const abc_stream* st)
{
    ABC_REQUIRE(st != nullptr, "stream selector is NULL");
    ABC_REQUIRE(st->domain <= 15u, "stream domain %u > 15", st->domain);
    return ABC_OK;
}

inline abc_status check_series(const abc_series* ser, bool need_obs)
{
    ABC_REQUIRE(ser != nullptr, "series is NULL");
    ABC_REQUIRE(ser->T >= 1 && ser->T <= ABC_T_MAX, "T = %d outside [1, %d]", ser->T, ABC_T_MAX);
    ABC_REQUIRE(ser->A0 >= 1 && ser->R0 >= 0 && ser->D0 >= 0, "need A0 >= 1, R0 >= 0, D0 >= 0");
    ABC_REQUIRE(ser->P <= INT32_MAX, "P = %lld does not fit the int32 state", (long long)ser->P);
    ABC_REQUIRE((int64_t)ser->A0 + ser->R0 + ser->D0 <= ser->P,
                "A0 + R0 + D0 exceeds the population P");
    if (need_obs) ABC_REQUIRE(ser->obs != nullptr, "series obs is NULL");
    return ABC_OK;
}

inline abc_status check_model(const abc_model* m)
{
    ABC_REQUIRE(m != nullptr, "model is NULL");
    ABC_REQUIRE(isfinite(m->noise_scale) && m->noise_scale >= 0.0f, "noise_scale must be finite and >= 0");
    ABC_REQUIRE((m->flags & ~(ABC_FP64 | ABC_KAHAN | ABC_NOISE_LITERAL | ABC_DIST_RAW | ABC_SUPPORT |
                               ABC_NO_BOUND)) == 0u,
                "unknown model flags 0x%x", m->flags);
    return ABC_OK;
}

}  // namespace abc
