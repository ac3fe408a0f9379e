// metropolis.hpp -- bit-sliced checkerboard Metropolis update of one site for
// 64 replicas at once.
//
// A 64-bit word holds one site of 64 consecutive replicas (bit b = replica
// 64g + b; a set bit is spin -1).  For the site's four bonds the word
// d_k = s ^ s_k ^ j_k has bit b set where the bond is unsatisfied
// (J s s_k = -1).  With u = number of unsatisfied bonds the energy change of
// a flip is dE = 2 s h = 8 - 4u: u >= 2 means dE <= 0 (always flip), u = 1
// means dE = +4 and u = 0 means dE = +8 (flip iff the replica's 32-bit draw
// is below the threshold T(beta_i, dE)).
//
// The draw of replica b is the 32-bit number whose bit 31-p is bit b of bit
// plane p; Philox call c (counter (n | c << 20, g, i, tag)) yields planes 2c
// (o0 | o1 << 32) and 2c + 1 (o2 | o3 << 32).  Comparing u < T most
// significant bit first, a lane is decided at the first plane where its bit
// differs from T's bit (accept if T's bit is 1).  Planes are generated only
// while some lane of the word is undecided; the result is identical to the
// full 32-bit comparison.
#pragma once

#include "philox.hpp"

namespace pa {

struct Thresholds {
    uint32_t t4, t8;        // low 32 bits of T(beta, 4), T(beta, 8)
    bool all4, all8;        // T == 2^32: every such move is accepted
};

constexpr int LUT_SEL = lut3((LUT_A & LUT_B) | (~LUT_A & LUT_C));   // a ? b : c, bitwise
constexpr int LUT_WIN = lut3(LUT_A & LUT_B & ~LUT_C);               // a & b & ~c
constexpr int LUT_TIE = lut3(LUT_A & ~(LUT_B ^ LUT_C));             // a & ~(b ^ c)
constexpr int LUT_NOR3 = lut3(~(LUT_A | LUT_B | LUT_C));
constexpr int LUT_ONE = lut3((LUT_A ^ LUT_B) & ~LUT_C);             // (a ^ b) & ~c
constexpr int LUT_OR_AND = lut3((LUT_A | LUT_B) & LUT_C);           // (a | b) & c

// Site classes of 64 replicas: flip = dE <= 0 (always flips), one = dE = +4,
// zero = dE = +8, from the word w, its four neighbours and the coupling
// masks (all ones where J = -1).
struct SiteClass {
    uint64_t flip, one, zero;
};

template <bool EA>
__device__ __forceinline__ SiteClass classify(uint64_t w, uint64_t nr, uint64_t nl, uint64_t nd, uint64_t nu,
                                              uint64_t jr, uint64_t jl, uint64_t jd, uint64_t ju)
{
    uint64_t d0, d1, d2, d3;
    if (EA) {
        d0 = bop3<LUT_XOR3>(w, nr, jr);
        d1 = bop3<LUT_XOR3>(w, nl, jl);
        d2 = bop3<LUT_XOR3>(w, nd, jd);
        d3 = bop3<LUT_XOR3>(w, nu, ju);
    } else {
        d0 = w ^ nr;
        d1 = w ^ nl;
        d2 = w ^ nd;
        d3 = w ^ nu;
    }
    const uint64_t x1 = d0 ^ d1, a1 = d0 & d1;
    const uint64_t x2 = d2 ^ d3, a2 = d2 & d3;
    SiteClass c;
    c.zero = bop3<LUT_NOR3>(d0, d1, d2) & ~d3;      // no unsatisfied bond
    c.one = bop3<LUT_ONE>(x1, x2, a1) & ~a2;        // exactly one
    c.flip = ~(c.zero | c.one);                     // two or more
    return c;
}

// One bit plane of the most-significant-first comparison u < T for the
// undecided lanes `und`: tb is T's bit for each lane's class (dE = +4 lanes
// where `one` is set, dE = +8 lanes elsewhere); a lane whose draw bit is 0
// where tb is 1 is accepted, a lane whose bits differ otherwise is rejected,
// equal bits stay undecided.
__device__ __forceinline__ void plane_step(uint64_t plane, uint64_t one, uint64_t m4, uint64_t m8,
                                           uint64_t &und, uint64_t &acc)
{
    const uint64_t tb = bop3<LUT_SEL>(one, m4, m8);
    acc |= bop3<LUT_WIN>(und, tb, plane);
    und = bop3<LUT_TIE>(und, tb, plane);
}

// Philox call c of a site: planes 2c and 2c+1 compared against T.
__device__ __forceinline__ void draw_step(uint32_t c, const Thresholds &T, uint64_t one, uint64_t &und,
                                          uint64_t &acc, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
    const u32x4 o = philox10(c0 | (c << 20), c1, c2, c3, k0, k1);
    const int sh = 31 - 2 * (int)c;
    const uint64_t m4a = (T.t4 >> sh) & 1u ? ~0ull : 0ull, m8a = (T.t8 >> sh) & 1u ? ~0ull : 0ull;
    const uint64_t m4b = (T.t4 >> (sh - 1)) & 1u ? ~0ull : 0ull, m8b = (T.t8 >> (sh - 1)) & 1u ? ~0ull : 0ull;
    plane_step((uint64_t)o.x | ((uint64_t)o.y << 32), one, m4a, m8a, und, acc);
    plane_step((uint64_t)o.z | ((uint64_t)o.w << 32), one, m4b, m8b, und, acc);
}

// Flip mask of one site, all draws done here (used by the plain path).
__device__ __forceinline__ uint64_t flip_mask(uint64_t w, uint64_t nr, uint64_t nl, uint64_t nd,
                                              uint64_t nu, uint64_t jr, uint64_t jl, uint64_t jd,
                                              uint64_t ju, const Thresholds &T, uint64_t valid,
                                              uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t &calls)
{
    SiteClass sc = classify<true>(w, nr, nl, nd, nu, jr, jl, jd, ju);
    if (T.all4) { sc.flip |= sc.one; sc.one = 0; }
    if (T.all8) { sc.flip |= sc.zero; sc.zero = 0; }
    uint64_t und = (sc.one | sc.zero) & valid;
    uint64_t acc = 0;
    for (uint32_t c = 0; und != 0 && c < 16; ++c) {
        draw_step(c, T, sc.one, und, acc, c0, c1, c2, c3, k0, k1);
        ++calls;
    }
    return sc.flip | acc;
}

__device__ __forceinline__ Thresholds thresholds_of(const uint64_t *tabT, int i)
{
    Thresholds T;
    const uint64_t a = tabT[2 * i], b = tabT[2 * i + 1];
    T.t4 = (uint32_t)a;
    T.t8 = (uint32_t)b;
    T.all4 = a >= (1ull << 32);
    T.all8 = b >= (1ull << 32);
    return T;
}

// Sign bits of 64 int8 spins (+1 = 0x01, -1 = 0xFF) packed into one word:
// bit b = 1 iff byte b is negative.
__device__ __forceinline__ uint32_t signs4(uint32_t d)
{
    return ((d >> 7) & 1u) | ((d >> 14) & 2u) | ((d >> 21) & 4u) | ((d >> 28) & 8u);
}

__device__ __forceinline__ uint64_t pack64(const uint4 v[4])
{
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        lo |= signs4(v[q].x) << (16 * q) | signs4(v[q].y) << (16 * q + 4) |
              signs4(v[q].z) << (16 * q + 8) | signs4(v[q].w) << (16 * q + 12);
        hi |= signs4(v[q + 2].x) << (16 * q) | signs4(v[q + 2].y) << (16 * q + 4) |
              signs4(v[q + 2].z) << (16 * q + 8) | signs4(v[q + 2].w) << (16 * q + 12);
    }
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// XOR mask that negates the bytes whose bit is set in the 4-bit group f4:
// 0x01 <-> 0xFF is an XOR with 0xFE.
__device__ __forceinline__ uint32_t negmask4(uint32_t f4)
{
    const uint32_t e = (f4 & 1u) | ((f4 & 2u) << 7) | ((f4 & 4u) << 14) | ((f4 & 8u) << 21);
    return (e << 8) - (e << 1);
}

__device__ __forceinline__ void apply64(uint4 v[4], uint64_t F)
{
    const uint32_t lo = (uint32_t)F, hi = (uint32_t)(F >> 32);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        v[q].x ^= negmask4((lo >> (16 * q)) & 15u);
        v[q].y ^= negmask4((lo >> (16 * q + 4)) & 15u);
        v[q].z ^= negmask4((lo >> (16 * q + 8)) & 15u);
        v[q].w ^= negmask4((lo >> (16 * q + 12)) & 15u);
        v[q + 2].x ^= negmask4((hi >> (16 * q)) & 15u);
        v[q + 2].y ^= negmask4((hi >> (16 * q + 4)) & 15u);
        v[q + 2].z ^= negmask4((hi >> (16 * q + 8)) & 15u);
        v[q + 2].w ^= negmask4((hi >> (16 * q + 12)) & 15u);
    }
}

}  // namespace pa
