// philox.hpp -- Philox4x32-10 counter-based generator for the GPU kernels.
//
// Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
// 3" (SC'11).  Ten rounds; per round the two even counter words are
// multiplied by fixed odd constants, the high halves of the 64-bit products
// are mixed with the odd words and the key, and the words are permuted; the
// key advances by two Weyl constants between rounds.
//
// gfx950 specifics: each 32x32->64 product is one v_mad_u64_u32, and each
// three-way XOR is one v_bitop3_b32, so a round is 2 + 2 VALU instructions.
// The key is the run (or disorder) seed and is uniform across a workgroup,
// so the key schedule lives in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

struct u32x4 {
    uint32_t x, y, z, w;
};

// Truth table of a three-input bitwise function f(a, b, c) for v_bitop3:
// f evaluated on the operand patterns a = 0xF0, b = 0xCC, c = 0xAA.
constexpr uint32_t LUT_A = 0xF0u, LUT_B = 0xCCu, LUT_C = 0xAAu;
constexpr int lut3(uint32_t v) { return (int)(v & 0xFFu); }

template <int LUT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, LUT);
}

template <int LUT>
__device__ __forceinline__ uint64_t bop3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, LUT);
    const uint32_t hi =
        __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), LUT);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

constexpr int LUT_XOR3 = lut3(LUT_A ^ LUT_B ^ LUT_C);   // 0x96

// Rounds FIRST .. 9 of Philox4x32-10 on counter (c0..c3) with the key of
// round FIRST.
template <int FIRST>
__device__ __forceinline__ u32x4 philox10_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1)
{
#pragma unroll
    for (int round = FIRST; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        if (round == 9) {
            // Keep the last products whole: otherwise the compiler may split
            // them into separate 32-bit low and high multiplies, which issue
            // at a quarter of the rate of one v_mad_u64_u32.  (An empty
            // statement that only pins the value in a register pair.)
            asm volatile("" : "+v"(p0));
            asm volatile("" : "+v"(p1));
        }
        const uint32_t n0 = bop3<LUT_XOR3>((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = bop3<LUT_XOR3>((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1)
{
    return philox10_rounds<0>(c0, c1, c2, c3, k0, k1);
}

// The same generator for the Metropolis draws: there the odd counter words
// of round 0 (the replica group and the tag word) and of round 1 (the low
// half of the product of the temperature index) are the same for every call
// of a site and often for the whole workgroup, so they are mixed with the key
// first, as a separate XOR that the compiler moves out of the call loops;
// rounds 2-9 are those of philox10.  (A chain of independent calls, as in the
// calibration, is better served by philox10's three-input XORs.)
__device__ __forceinline__ u32x4 philox10_sweep(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        const uint32_t x1 = c1 ^ k0, x3 = c3 ^ k1;
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(p1 >> 32) ^ x1;
        c2 = (uint32_t)(p0 >> 32) ^ x3;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    const u32x4 r = philox10_rounds<2>(c0, c1, c2, c3, k0, k1);
    return r;
}

}  // namespace pa
