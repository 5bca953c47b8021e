// Device Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011) specialised for the two counters the sampler
// uses.  Key = (seed, attempt id).  Every round multiplies the even counter
// words by the two Philox multipliers (full 128-bit products), xors the high
// halves with the odd words and the round key, and permutes; the key is bumped
// by the Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sia {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Word 0 of the block with counter (c0, c1, 0, 0) under key (k0, k1).
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t k0,
                                                 uint64_t k1)
{
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 128-bit product per multiplier: its halves share the partial
        // products (fewer 32-bit multiplies than separate high / low parts)
        const unsigned __int128 p0 = static_cast<unsigned __int128>(kPhiloxM0) * x0;
        const unsigned __int128 p1 = static_cast<unsigned __int128>(kPhiloxM1) * x2;
        const uint64_t y0 = static_cast<uint64_t>(p1 >> 64) ^ x1 ^ k0;
        const uint64_t y2 = static_cast<uint64_t>(p0 >> 64) ^ x3 ^ k1;
        x0 = y0;
        x1 = static_cast<uint64_t>(p1);
        x2 = y2;
        x3 = static_cast<uint64_t>(p0);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return x0;
}

// 32-bit draw that picks the live in-edge of node x in attempt a.
__device__ __forceinline__ uint32_t node_draw(uint64_t seed, uint64_t a, uint32_t x)
{
    return static_cast<uint32_t>(philox_word0(x, 0, seed, a) >> 32);
}

// 64-bit start draw of attempt a.
__device__ __forceinline__ uint64_t start_draw(uint64_t seed, uint64_t a)
{
    return philox_word0(0, 1, seed, a);
}

}  // namespace sia
