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

constexpr int LUT_ACCEPT = lut3(LUT_A & ~LUT_B & LUT_C);           // und & ~plane & m
constexpr int LUT_KEEP = lut3(LUT_A & ~(LUT_B ^ LUT_C));             // und & ~(plane ^ m)
constexpr int LUT_OR3 = lut3(LUT_A | LUT_B | LUT_C);

// One bit plane of the most-significant-first comparison u < T for the
// undecided lanes of both classes (dE = +4 in und4, dE = +8 in und8).  m4
// and m8 are all ones where T's bit at this plane is 1 for that class, and
// the same for the whole wavefront.  A lane whose draw bit differs from T's
// bit is decided (accepted iff T's bit is 1); equal bits stay undecided.
// Five three-input operations per 32 bits, each with one scalar operand.
__device__ __forceinline__ void plane_both(uint64_t plane, uint32_t m4, uint32_t m8, uint64_t &und4,
                                           uint64_t &und8, uint64_t &acc)
{
    const uint32_t p[2] = {(uint32_t)plane, (uint32_t)(plane >> 32)};
    uint32_t u4[2] = {(uint32_t)und4, (uint32_t)(und4 >> 32)};
    uint32_t u8[2] = {(uint32_t)und8, (uint32_t)(und8 >> 32)};
    uint32_t a[2] = {(uint32_t)acc, (uint32_t)(acc >> 32)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t x4 = bop3<LUT_ACCEPT>(u4[h], p[h], m4);
        const uint32_t x8 = bop3<LUT_ACCEPT>(u8[h], p[h], m8);
        a[h] = bop3<LUT_OR3>(a[h], x4, x8);
        u4[h] = bop3<LUT_KEEP>(u4[h], p[h], m4);
        u8[h] = bop3<LUT_KEEP>(u8[h], p[h], m8);
    }
    und4 = (uint64_t)u4[0] | ((uint64_t)u4[1] << 32);
    und8 = (uint64_t)u8[0] | ((uint64_t)u8[1] << 32);
    acc = (uint64_t)a[0] | ((uint64_t)a[1] << 32);
}

// Philox call c of a site: planes 2c and 2c+1 compared against the
// thresholds t4 = T(beta, 4) and t8 = T(beta, 8) (low 32 bits; both
// wavefront-uniform), for the undecided lanes of each class.
__device__ __forceinline__ void draw_call(uint32_t c, uint32_t t4, uint32_t t8, uint64_t &und4, uint64_t &und8,
                                          uint64_t &acc, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
    const u32x4 o = philox10_sweep(c0 | (c << 20), c1, c2, c3, k0, k1);
    const uint32_t sh = 31u - 2u * c;
    const uint64_t pa = (uint64_t)o.x | ((uint64_t)o.y << 32);
    const uint64_t pb = (uint64_t)o.z | ((uint64_t)o.w << 32);
    plane_both(pa, 0u - ((t4 >> sh) & 1u), 0u - ((t8 >> sh) & 1u), und4, und8, acc);
    plane_both(pb, 0u - ((t4 >> (sh - 1u)) & 1u), 0u - ((t8 >> (sh - 1u)) & 1u), und4, und8, acc);
}

// T's bits at the planes of call c as all-ones or zero masks: x = plane 2c
// (bit 31 - 2c), y = plane 2c + 1 (bit 30 - 2c), for dE = +4 (x, y) and
// +8 (z, w).
__device__ __forceinline__ uint4 call_masks(uint32_t t4, uint32_t t8, uint32_t c)
{
    const uint32_t sh = 31u - 2u * c;
    return make_uint4(0u - ((t4 >> sh) & 1u), 0u - ((t4 >> (sh - 1u)) & 1u), 0u - ((t8 >> sh) & 1u),
                      0u - ((t8 >> (sh - 1u)) & 1u));
}

// draw_call for a call index c that differs between lanes, with T's bits
// at its planes given as masks (call_masks of each lane's c).
__device__ __forceinline__ void draw_call_masks(uint32_t c, uint4 m, uint64_t &und4, uint64_t &und8, uint64_t &acc,
                                                uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1)
{
    const u32x4 o = philox10_sweep(c0 | (c << 20), c1, c2, c3, k0, k1);
    const uint64_t pa = (uint64_t)o.x | ((uint64_t)o.y << 32);
    const uint64_t pb = (uint64_t)o.z | ((uint64_t)o.w << 32);
    plane_both(pa, m.x, m.z, und4, und8, acc);
    plane_both(pb, m.y, m.w, und4, und8, acc);
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
    uint64_t und4 = sc.one & valid, und8 = sc.zero & valid;
    uint64_t acc = sc.flip;
    for (uint32_t c = 0; (und4 | und8) != 0 && c < 16; ++c) {
        draw_call(c, T.t4, T.t8, und4, und8, acc, c0, c1, c2, c3, k0, k1);
        ++calls;
    }
    return acc;
}

// Thresholds of temperature i, read once per workgroup and kept in scalar
// registers.
__device__ __forceinline__ Thresholds thresholds_of(const uint64_t *tabT, int i)
{
    Thresholds T;
    const uint64_t a = tabT[2 * i], b = tabT[2 * i + 1];
    T.t4 = __builtin_amdgcn_readfirstlane((uint32_t)a);
    T.t8 = __builtin_amdgcn_readfirstlane((uint32_t)b);
    T.all4 = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) != 0;
    T.all8 = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) != 0;
    return T;
}

// Sign bits of 16 int8 spins (+1 = 0x01, -1 = 0xFF; four bytes per 32-bit
// lane of v, byte k of v.x first): bit k = 1 iff byte k is negative.  Each
// byte's bit 7 is isolated (0x80 or 0) and weighted by a power of two in an
// unsigned 4-byte dot product, so two dwords give 128 x (their 8 bits).
__device__ __forceinline__ uint32_t signs16(const uint4 &v)
{
    uint32_t lo = __builtin_amdgcn_udot4(v.x & 0x80808080u, 0x08040201u, 0u, false);
    lo = __builtin_amdgcn_udot4(v.y & 0x80808080u, 0x80402010u, lo, false);
    uint32_t hi = __builtin_amdgcn_udot4(v.z & 0x80808080u, 0x08040201u, 0u, false);
    hi = __builtin_amdgcn_udot4(v.w & 0x80808080u, 0x80402010u, hi, false);
    return (lo >> 7) | ((hi >> 7) << 8);
}

__device__ __forceinline__ uint64_t pack64(const uint4 v[4])
{
    return (uint64_t)(signs16(v[0]) | (signs16(v[1]) << 16)) |
           ((uint64_t)(signs16(v[2]) | (signs16(v[3]) << 16)) << 32);
}

// Four canonical spin bytes from 4 sign bits f4 (bit k set: byte k = 0xFF,
// else 0x01).  The multiply by 2^0 + 2^7 + 2^14 + 2^21 moves bit k to bit 8k
// among terms at pairwise distinct positions (no carries); each selected bit
// then becomes 0xFE + 0x01 in its byte.
__device__ __forceinline__ uint32_t spins4(uint32_t f4)
{
    const uint32_t e = (f4 * 0x00204081u) & 0x01010101u;
    return e * 0xFEu + 0x01010101u;
}

// 16 canonical spin bytes from 16 sign bits (the inverse of signs16).
__device__ __forceinline__ uint4 spins16(uint32_t b)
{
    uint4 v;
    v.x = spins4(b & 15u);
    v.y = spins4((b >> 4) & 15u);
    v.z = spins4((b >> 8) & 15u);
    v.w = spins4((b >> 12) & 15u);
    return v;
}

}  // namespace pa
