// Error reporting and version of libabc.so.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>

#include "common.hpp"

namespace abc {

static thread_local char g_last_error[512] = "";

// The message is formatted into a temporary first, so that an argument may be
// the previous message itself (abc_last_error(), to prefix it with context).
abc_status set_error(abc_status st, const char* fmt, ...)
{
    char buf[sizeof g_last_error];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    memcpy(g_last_error, buf, sizeof buf);
    return st;
}

constexpr int INFO_MAX_DEVICES = 64;
static std::mutex g_info_mu;
static DeviceInfo g_info[INFO_MAX_DEVICES];

abc_status device_info(DeviceInfo* out)
{
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    ABC_REQUIRE(dev >= 0 && dev < INFO_MAX_DEVICES, "device %d beyond the library's %d", dev,
                INFO_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_info_mu);
    DeviceInfo& d = g_info[dev];
    if (d.num_cu == 0) {
        ABC_HIP(hipDeviceGetAttribute(&d.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        ABC_HIP(hipDeviceGetAttribute(&d.num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    *out = d;
    return ABC_OK;
}

struct ScratchKey {
    int dev;
    hipStream_t stream;
    int slot;
    bool operator<(const ScratchKey& o) const
    {
        if (dev != o.dev) return dev < o.dev;
        if (stream != o.stream) return (uintptr_t)stream < (uintptr_t)o.stream;
        return slot < o.slot;
    }
};
struct ScratchBuf {
    void* p = nullptr;
    size_t bytes = 0;
};
static std::mutex g_scratch_mu;
static std::map<ScratchKey, ScratchBuf> g_scratch;

abc_status stream_scratch(hipStream_t s, size_t bytes, void** out, int slot)
{
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    if (bytes == 0) bytes = 256;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchBuf& b = g_scratch[ScratchKey{dev, s, slot}];
    if (b.bytes < bytes) {
        // round up so that a few growing requests settle quickly
        size_t want = 1u << 16;
        while (want < bytes) want <<= 1;
        if (b.p) {
            ABC_HIP(hipStreamSynchronize(s));  // earlier work on s may still use it
            ABC_HIP(hipFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
        }
        const hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            b.p = nullptr;
            return set_error(ABC_ENOMEM, "scratch of %zu B: %s", want, hipGetErrorString(e));
        }
        b.bytes = want;
    }
    *out = b.p;
    return ABC_OK;
}

static std::map<ScratchKey, ScratchBuf> g_pinned;

abc_status stream_pinned(hipStream_t s, size_t bytes, void** out)
{
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    if (bytes == 0) bytes = 64;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchBuf& b = g_pinned[ScratchKey{dev, s, 0}];
    if (b.bytes < bytes) {
        size_t want = 4096;
        while (want < bytes) want <<= 1;
        if (b.p) {
            ABC_HIP(hipStreamSynchronize(s));
            ABC_HIP(hipHostFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
        }
        const hipError_t e = hipHostMalloc(&b.p, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            b.p = nullptr;
            return set_error(ABC_ENOMEM, "pinned scratch of %zu B: %s", want, hipGetErrorString(e));
        }
        b.bytes = want;
    }
    *out = b.p;
    return ABC_OK;
}

}  // namespace abc

extern "C" abc_status abc_release_scratch(void)
{
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    ABC_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lock(abc::g_scratch_mu);
    for (auto it = abc::g_scratch.begin(); it != abc::g_scratch.end();) {
        if (it->first.dev == dev) {
            if (it->second.p) ABC_HIP(hipFree(it->second.p));
            it = abc::g_scratch.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = abc::g_pinned.begin(); it != abc::g_pinned.end();) {
        if (it->first.dev == dev) {
            if (it->second.p) ABC_HIP(hipHostFree(it->second.p));
            it = abc::g_pinned.erase(it);
        } else {
            ++it;
        }
    }
    return ABC_OK;
}

extern "C" const char* abc_last_error(void) { return abc::g_last_error; }

extern "C" const char* abc_version(void) { return "abc-mi355x 0.1 (gfx950)"; }
