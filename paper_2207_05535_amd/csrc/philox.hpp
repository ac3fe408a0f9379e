// philox.hpp -- Philox4x32-10 counter-based generator for the GPU kernels.
//
// Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
// 3" (SC'11).  Ten rounds; per round the two even counter words are
// multiplied by fixed odd constants, the high halves of the 64-bit products
// are mixed with the odd words and the key, and the words are permuted; the
// key advances by two Weyl constants between rounds.  The key is the run (or
// disorder) seed and is uniform across a workgroup, so the key schedule
// lives in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

}  // namespace pa
