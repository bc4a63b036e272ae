// philox.hpp -- the counter-based generator Philox4x64-10 (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), from
// its published definition: ten rounds of two 64x64 -> 128-bit products with
// the published multipliers, the key bumped by the published Weyl constants
// between rounds; and the map of a 64-bit word to a uniform in (0,1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msg {

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double uniform52(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

}  // namespace msg
