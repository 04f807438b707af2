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

constexpr uint32_t PH_M0 = 0xD2511F53u;
constexpr uint32_t PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u;
constexpr uint32_t PH_W1 = 0xBB67AE85u;

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox_round(uint4 c, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)c.z;
    return make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                      xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, Key key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        c = philox_round(c, k0, k1);
        k0 += PH_W0;
        k1 += PH_W1;
    }
    return c;
}

// Day-loop form of the generator for one sample. In the counter
// (i_lo, i_hi, series, w) only w changes from day to day, so part of rounds
// 1-3 is fixed per sample: begin() computes it once (three products), and
// day(w) finishes the remaining 16 products.
struct PhiloxDays {
    uint32_t c1base;  // hi(M0 i_lo) ^ k1
    uint32_t g3;      // hi(M1 e2) ^ k0 + 2 W0, e2 = round-2 word z
    uint32_t h3;      // lo(M1 e2)
    uint32_t f3;      // round-2 word w ^ (k1 + 2 W1)

    // u0 = hi(M1 series) ^ k0 (wave-uniform)
    __device__ __forceinline__ void begin(uint64_t i, uint32_t u0, Key key)
    {
        const uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)(uint32_t)i;
        c1base = (uint32_t)(p0 >> 32) ^ key.k1;
        const uint32_t d1 = (uint32_t)p0;
        const uint32_t a1 = u0 ^ (uint32_t)(i >> 32);
        const uint64_t q0 = (uint64_t)PH_M0 * (uint64_t)a1;
        const uint32_t e2 = xor3((uint32_t)(q0 >> 32), d1, key.k1 + PH_W1);
        const uint32_t f2 = (uint32_t)q0;
        const uint64_t r1 = (uint64_t)PH_M1 * (uint64_t)e2;
        g3 = (uint32_t)(r1 >> 32) ^ (key.k0 + 2u * PH_W0);
        h3 = (uint32_t)r1;
        f3 = f2 ^ (key.k1 + 2u * PH_W1);
    }

    // b1 = lo(M1 series) ^ (k0 + W0) (wave-uniform); w = fourth counter word
    __device__ __forceinline__ uint4 day(uint32_t w, uint32_t b1, Key key) const
    {
        const uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)(c1base ^ w);
        const uint32_t x2 = (uint32_t)(p1 >> 32) ^ b1;
        const uint32_t y2 = (uint32_t)p1;
        const uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)x2;
        uint4 c = make_uint4(g3 ^ y2, h3, (uint32_t)(p0 >> 32) ^ f3, (uint32_t)p0);
#pragma unroll
        for (int r = 3; r < 10; ++r)
            c = philox_round(c, key.k0 + (uint32_t)r * PH_W0, key.k1 + (uint32_t)r * PH_W1);
        return c;
    }
};

// Wave-uniform parts of the day form for one series.
struct PhiloxSeries {
    uint32_t u0, b1;
};

__device__ __forceinline__ PhiloxSeries philox_series(uint32_t series, Key key)
{
    const uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)series;
    return PhiloxSeries{(uint32_t)(p1 >> 32) ^ key.k0, (uint32_t)p1 ^ (key.k0 + PH_W0)};
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
