// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11) and the stream layout of this
// library: key = (seed mod 2^32, seed >> 32), counter = (i mod 2^32, i >> 32,
// series, day << 8 | domain << 4 | block).
//
// On gfx950 each round is two 32x32->64 products (v_mad_u64_u32) and two
// three-way XORs; the key schedule is wave-uniform and stays in SGPRs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abc {

struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, Key key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__host__ __device__ __forceinline__ Key make_key(uint64_t seed)
{
    return Key{(uint32_t)seed, (uint32_t)(seed >> 32)};
}

// Fourth counter word for (day, domain, block).
__host__ __device__ __forceinline__ uint32_t ctr_word3(uint32_t day, uint32_t domain, uint32_t block)
{
    return (day << 8) | (domain << 4) | block;
}

__device__ __forceinline__ uint4 stream_words(Key key, uint64_t sample, uint32_t series,
                                              uint32_t w3)
{
    return philox4x32_10(make_uint4((uint32_t)sample, (uint32_t)(sample >> 32), series, w3), key);
}

}  // namespace abc
