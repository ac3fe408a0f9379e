// kernels.hip -- HIP kernels of the population-annealing temperature step
// for gfx950 (CDNA4, 64-wide wavefronts).
//
// Step (i)   k_init_couplings, k_init_spins, k_init_fam (Sec. II B, III A)
// Step (ii)  k_rw_chunk, k_rw_finish                   (Eqs. (QBoltz), (F))
// Step (iii) k_cnt_chunk, k_mn_draws, k_cnt_scan_chunk, k_cnt_finish,
//            k_parent, k_copy                          (Sec. II B, IV D, V A 1)
// Step (iv)  k_sweep_int8 (one colour of one run per launch),
//            k_sweep_msc (all runs, lattice in LDS for all theta sweeps;
//            also compiled per lattice size and model), k_dos_sample (the
//            theta = infinity limit, Sec. V C)
// Step (v)   k_wang_pairs, k_wang_rows, k_wang_gather (permutation pairing,
//            Sec. III D), k_measure, k_meas_chunk, k_finalize
//                                                      (Eqs. (e)-(chi), Sec. III D)
// Sec. IV    k_logw, k_qweights, k_wavg, k_wavg_cumsum, k_wqhist, k_famstats
// Diagnostic k_philox_rate (integer-VALU calibration)
//
// Population-wide reductions and scans are split into fixed-size chunks of
// CH replicas (one workgroup each) plus a single-workgroup pass over the
// chunk totals, so every result is independent of the launch shape and the
// floating-point sums have one fixed order.
#include <float.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <queue>
#include <type_traits>
#include <vector>
#include <math.h>
#include <stdint.h>

#include "launch.hpp"
#include "metropolis.hpp"
#include "pa_internal.hpp"
#include "philox.hpp"

namespace pa {

// Index of this thread's wavefront in the workgroup, as a value the compiler
// knows to be uniform in the wavefront (loop bounds and counts derived from it
// then stay in scalar registers).
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// ------------------------------------------------------------- utilities

__device__ __forceinline__ uint64_t umul64hi(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// floor(rem * 2^32 / d) for rem < d < 2^63: 32 steps of binary long division.
__device__ __forceinline__ uint32_t frac32(uint64_t rem, uint64_t d)
{
    uint32_t q = 0;
#pragma unroll 4
    for (int k = 0; k < 32; ++k) {
        rem <<= 1;
        q <<= 1;
        if (rem >= d) {
            rem -= d;
            q |= 1u;
        }
    }
    return q;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ bool pop_active(const PopState &S) { return S.moved && S.status == PA_OK; }

// Value of lane (lane ^ J) for a 32-bit register, with the cheapest gfx950
// cross-lane form for each distance: permlane swaps for 32 and 16, an LDS
// swizzle for 8 and 4, DPP quad permutes for 2 and 1.
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    if constexpr (J == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else if constexpr (J == 8 || J == 4) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1f);
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    }
}

// One block-swap stage of the transpose for J < 32, on each 32-bit half:
// m holds the bit positions without bit J.  A lane without bit J keeps
// those and sends the others, moved down by J; its partner (lane ^ J) keeps
// the others and sends those, moved up by J.  Both moves are one rotation
// (right by J, or by 32 - J) followed by the kept-bits mask, since the bits
// that wrap around land outside it; no branch on the lane's side.
template <int J>
__device__ __forceinline__ void transpose_stage(uint32_t &lo, uint32_t &hi, uint32_t m)
{
    const uint32_t up = 0u - ((threadIdx.x / J) & 1u);   // all ones on lanes with bit J
    const uint32_t keep = m ^ up;
    const uint32_t sh = J + (up & (32u - 2u * J));
    const uint32_t slo = __builtin_amdgcn_alignbit(lo, lo, sh) & keep;
    const uint32_t shi = __builtin_amdgcn_alignbit(hi, hi, sh) & keep;
    lo = (lo & keep) | lane_xor<J>(slo);
    hi = (hi & keep) | lane_xor<J>(shi);
}

// 64 x 64 bit transpose across a wavefront: lane r holds row r (bit c =
// element (r, c)); on return lane r holds column r.  Six block-swap stages
// (distances 32, 16, 8, 4, 2, 1): the first exchanges one 32-bit half, the
// others exchange within each half.
__device__ __forceinline__ uint64_t transpose64(uint64_t x)
{
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {
        const bool up = threadIdx.x & 32;
        const uint32_t r = lane_xor<32>(up ? lo : hi);
        lo = up ? r : lo;
        hi = up ? hi : r;
    }
    transpose_stage<16>(lo, hi, 0x0000FFFFu);
    transpose_stage<8>(lo, hi, 0x00FF00FFu);
    transpose_stage<4>(lo, hi, 0x0F0F0F0Fu);
    transpose_stage<2>(lo, hi, 0x33333333u);
    transpose_stage<1>(lo, hi, 0x55555555u);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Bit-sliced (vertical) counters: plane k holds bit k of 64 per-lane counts.
constexpr int VB = 6;   // counts up to 63 per lane

// Carry-save counting of a block of 16 sites per lane, Harley and Seal's
// scheme in bit-sliced form: a three-input adder (sum = XOR, carry =
// majority, one bitop3 each per 32 bits) folds each site's inputs into the
// ones plane and passes its carry up; carries of equal weight wait for a
// partner from a later site, so after the 16th site the planes ones, twos,
// fours, eights and the sixteens are the binary digits of every lane's count.
// The site index t (the same on every lane) decides which carries pair up;
// every block takes exactly the 16 sites t = 0 .. 15 in order (zero inputs
// for missing ones).
constexpr int LUT_MAJ3 = lut3((LUT_A & LUT_B) | (LUT_A & LUT_C) | (LUT_B & LUT_C));

__device__ __forceinline__ void csa(uint64_t &carry, uint64_t &sum, uint64_t a, uint64_t b, uint64_t c)
{
    const uint64_t s = bop3<LUT_XOR3>(a, b, c);
    carry = bop3<LUT_MAJ3>(a, b, c);
    sum = s;
}

// One input per site: counts up to 16 in five planes.
struct Csa1 {
    uint64_t p1 = 0, p2 = 0, p4 = 0, p8 = 0, p16 = 0, w1 = 0, w2 = 0, w4 = 0, w8 = 0;
    __device__ __forceinline__ void add(int t, uint64_t a)
    {
        if (!(t & 1)) { w1 = a; return; }
        uint64_t c2, c4, c8;
        csa(c2, p1, p1, w1, a);
        if (!(t & 2)) { w2 = c2; return; }
        csa(c4, p2, p2, w2, c2);
        if (!(t & 4)) { w4 = c4; return; }
        csa(c8, p4, p4, w4, c4);
        if (!(t & 8)) { w8 = c8; return; }
        csa(p16, p8, p8, w8, c8);
    }
    __device__ __forceinline__ void planes(uint64_t (&p)[VB]) const
    {
        p[0] = p1; p[1] = p2; p[2] = p4; p[3] = p8; p[4] = p16; p[5] = 0;
    }
};

// Two inputs per site: counts up to 32 in six planes.
struct Csa2 {
    uint64_t p1 = 0, p2 = 0, p4 = 0, p8 = 0, s16a = 0, s16b = 0, w2 = 0, w4 = 0, w8 = 0;
    __device__ __forceinline__ void add(int t, uint64_t a, uint64_t b)
    {
        uint64_t c2, c4, c8;
        csa(c2, p1, p1, a, b);
        if (!(t & 1)) { w2 = c2; return; }
        csa(c4, p2, p2, w2, c2);
        if (!(t & 2)) { w4 = c4; return; }
        csa(c8, p4, p4, w4, c4);
        if (!(t & 4)) { w8 = c8; return; }
        csa((t & 8) ? s16b : s16a, p8, p8, w8, c8);
    }
    __device__ __forceinline__ void planes(uint64_t (&p)[VB]) const
    {
        p[0] = p1; p[1] = p2; p[2] = p4; p[3] = p8; p[4] = s16a ^ s16b; p[5] = s16a & s16b;
    }
};

// Incremental form (a half-adder chain per input), used where fewer
// registers matter more than fewer operations.
__device__ __forceinline__ void vinc(uint64_t (&p)[VB], uint64_t x)
{
#pragma unroll
    for (int k = 0; k < VB; ++k) {
        const uint64_t t = p[k] & x;
        p[k] ^= x;
        x = t;
    }
}

// add the 2-bit per-lane values a + b
__device__ __forceinline__ void vinc2(uint64_t (&p)[VB], uint64_t a, uint64_t b)
{
    const uint64_t s = a ^ b, c = a & b;
    const uint64_t t0 = p[0] & s;
    p[0] ^= s;
    uint64_t x = t0 | c;
#pragma unroll
    for (int k = 1; k < VB; ++k) {
        const uint64_t t = p[k] & x;
        p[k] ^= x;
        x = t;
    }
}

// Per-lane counts summed over the wavefront: on return lane b holds the
// total over all lanes of bit b's count, and the planes are cleared.  Only
// the lowest `used` planes (wavefront-uniform) can be non-zero.
__device__ __forceinline__ uint32_t vflush(uint64_t (&p)[VB], int used = VB)
{
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < VB; ++k) {
        if (k < used) total += (uint32_t)__popcll(transpose64(p[k])) << k;
        p[k] = 0;
    }
    return total;
}

// Bit planes that hold counts up to c.
__device__ __forceinline__ int planes_for(int c) { return 32 - __clz(c); }

// Exclusive scan of one value per thread across a workgroup of BS threads
// (BS a multiple of 64); returns the exclusive prefix, *total the sum.
template <typename T, int BS>
__device__ __forceinline__ T block_exscan(T v, T *lds, T *total)
{
    const int lane = threadIdx.x & 63, wv = wave_id();
    T incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int k = 0; k < BS / 64; ++k) {
            T t = lds[k];
            lds[k] = run;
            run += t;
        }
        lds[BS / 64] = run;
    }
    __syncthreads();
    T res = lds[wv] + incl - v;
    *total = lds[BS / 64];
    __syncthreads();
    return res;
}

// ------------------------------------------------------------------ fill

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n)
{
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// -------------------------------------------------------------- step (i)

// Couplings of the +-J model: J_R(n) = -1 iff bit 0 of o0, J_D(n) = -1 iff
// bit 0 of o1, of Philox(disorder seed; n, 0, 0, TAG_J << 28).
__global__ void k_init_couplings(const RunInfo *runs, const uint64_t *dseed)
{
    const RunInfo &R = runs[blockIdx.x];
    const uint64_t ds = dseed[blockIdx.x];
    for (int n = threadIdx.x; n < R.N; n += blockDim.x) {
        uint8_t b = 0;
        if (R.model == PA_EA_PMJ) {
            const u32x4 o = philox10((uint32_t)n, 0, 0, TAG_J << 28, (uint32_t)ds, (uint32_t)(ds >> 32));
            b = (uint8_t)((o.x & 1u) | ((o.y & 1u) << 1));
        }
        R.jbits[n] = b;
    }
}

// Spins at beta_0 = 0: bit b of o0 | o1 << 32 of Philox(seed; n, g, 0,
// TAG_INIT << 28 | pop << 24) is replica 64 g + b at site n (set = -1).
template <int REPR>
__global__ void k_init_spins(const Item *items, const RunInfo *runs)
{
    const Item it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const uint32_t c3 = (TAG_INIT << 28) | ((uint32_t)it.pop << 24);
    for (int n = threadIdx.x; n < R.N; n += blockDim.x) {
        const u32x4 o = philox10((uint32_t)n, (uint32_t)it.group, 0, c3, R.key0, R.key1);
        const uint64_t plane = (uint64_t)o.x | ((uint64_t)o.y << 32);
        const size_t site = (size_t)it.group * R.N + n;
        if (REPR == PA_MSC64) {
            ((uint64_t *)R.spins[it.pop][0])[site] = plane;
        } else {
            uint4 *dst = (uint4 *)(R.spins[it.pop][0] + site * 64);
            for (int q = 0; q < 4; ++q) dst[q] = spins16((uint32_t)(plane >> (16 * q)) & 0xFFFFu);
        }
    }
}

__global__ void k_init_fam(const RunInfo *runs)
{
    const RunInfo &R = runs[blockIdx.x];
    for (int p = 0; p < R.npop; ++p)
        for (int j = threadIdx.x; j < R.R_cap; j += blockDim.x) {
            R.fam[p][0][j] = j < R.R ? j : 0;
            R.E[p][0][j] = 0;
        }
}

// ------------------------------------------------------------- step (ii)

// Reweighting, Eq. (tauBoltz)/(QBoltz): per chunk of CH replicas the partial
// sums of x_j = exp(-dbeta (E_j - E_min)) (FP64) and of X_j = floor(x_j 2^40)
// (exact); for multinomial resampling also the chunk-local exclusive prefix
// of X_j.  The temperature index is i = (index of the population) + 1.
__global__ void __launch_bounds__(CH_THREADS) k_rw_chunk(const ChunkItem *items, const RunInfo *runs,
                                                          const PopState *st)
{
    __shared__ uint64_t lds64[CH_THREADS / 64 + 1];
    __shared__ double ldsd[CH_THREADS / 64];
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (S.status != PA_OK) return;
    const int i = S.i + 1;
    if (i >= R.K) return;
    const int Rp = S.Rcur;
    const int j0 = it.chunk * CH;
    if (j0 >= Rp) return;
    const int32_t *E = R.E[it.pop][S.cur];
    const int Np1 = R.N + 1;
    const uint64_t *X = R.tabX + (size_t)i * Np1;
    const double *x = R.tabx + (size_t)i * Np1;
    const int Emin = S.Emin;
    // each thread: CH_PER consecutive replicas, summed in order
    const int jb = j0 + threadIdx.x * CH_PER;
    double s = 0.0;
    uint64_t sx = 0;
    uint64_t loc[CH_PER];
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        const int j = jb + q;
        uint64_t Xj = 0;
        if (j < Rp) {
            const int k = min(max((E[j] - Emin) >> 2, 0), R.N);
            Xj = X[k];
            s += x[k];
        }
        loc[q] = sx;
        sx += Xj;
    }
    uint64_t tot;
    const uint64_t pre = block_exscan<uint64_t, CH_THREADS>(sx, lds64, &tot);
    if (R.resampling == PA_MULTINOMIAL) {
        uint64_t *P = R.P[it.pop];
#pragma unroll
        for (int q = 0; q < CH_PER; ++q)
            if (jb + q < Rp) P[jb + q] = pre + loc[q];
    }
    // fixed-order FP64 tree: wave shuffles then waves in order
    double ws = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) ws += __shfl_xor(ws, o, 64);
    if ((threadIdx.x & 63) == 0) ldsd[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < CH_THREADS / 64; ++k) t += ldsd[k];
        R.partS[it.pop][it.chunk] = t;
        R.tot64[it.pop][it.chunk] = tot;
    }
}

// ln Q_i = ln S - ln R_{i-1} - dbeta E_min and A_i = A_{i-1} + ln Q_i,
// Eqs. (QBoltz), (F); chunk bases of the X prefix for multinomial draws.
__global__ void k_rw_finish(const RunInfo *runs, PopState *st)
{
    __shared__ uint64_t lds64[257];
    const int run = blockIdx.x, pop = blockIdx.y;
    const RunInfo &R = runs[run];
    if (pop >= R.npop) return;
    PopState &S = st[run * MAX_POP + pop];
    const int i = S.i + 1;
    const bool go = S.status == PA_OK && i < R.K;
    if (!go) {
        if (threadIdx.x == 0) S.moved = 0;
        return;
    }
    const int Rp = S.Rcur;
    const int nch = (Rp + CH - 1) / CH;
    uint64_t carry = 0;
    for (int base = 0; base < nch; base += 256) {
        const int c = base + threadIdx.x;
        const uint64_t v = c < nch ? R.tot64[pop][c] : 0;
        uint64_t tot;
        const uint64_t pre = block_exscan<uint64_t, 256>(v, lds64, &tot);
        if (c < nch) R.base64[pop][c] = carry + pre;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        double Ssum = 0.0;
        for (int c = 0; c < nch; ++c) Ssum += R.partS[pop][c];
        const double db = R.beta[i] - R.beta[i - 1];
        const double lnQ = log(Ssum) - log((double)Rp) - db * (double)S.Emin;
        S.lnQ = lnQ;
        S.A = S.A + lnQ;
        S.S = Ssum;
        S.SX = carry;
        S.Rprev = Rp;
        S.i = i;
        S.moved = 1;
    }
}

// ------------------------------------------------------------ step (iii)

// Nearest-integer counts r_j = n_j + [u_j < t_j], n_j = floor(R X_j / S_X),
// t_j = floor((R X_j mod S_X) 2^32 / S_X), u_j = o0 of Philox(seed; j, 0, i,
// TAG_NI << 28 | pop << 24); then the chunk-local exclusive prefix of r.
// For multinomial resampling this only clears r.
__global__ void __launch_bounds__(CH_THREADS) k_cnt_chunk(const ChunkItem *items, const RunInfo *runs,
                                                           const PopState *st)
{
    __shared__ int32_t lds[CH_THREADS / 64 + 1];
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rp = S.Rprev;
    const int j0 = it.chunk * CH;
    if (j0 >= Rp) return;
    const int jb = j0 + threadIdx.x * CH_PER;
    int32_t *r = R.r[it.pop];
    if (R.resampling == PA_MULTINOMIAL) {
#pragma unroll
        for (int q = 0; q < CH_PER; ++q)
            if (jb + q < Rp) r[jb + q] = 0;
        return;
    }
    const int i = S.i;
    const int32_t *E = R.E[it.pop][S.cur];
    const uint64_t *X = R.tabX + (size_t)i * (R.N + 1);
    const uint64_t SX = S.SX;
    const uint32_t c3 = (TAG_NI << 28) | ((uint32_t)it.pop << 24);
    int32_t loc[CH_PER];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        const int j = jb + q;
        int32_t rj = 0;
        if (j < Rp) {
            const uint64_t RX = (uint64_t)R.R * X[min(max((E[j] - S.Emin) >> 2, 0), R.N)];
            const uint64_t n = RX / SX;
            const uint64_t rem = RX - n * SX;
            const uint32_t t = frac32(rem, SX);
            const u32x4 o = philox10((uint32_t)j, 0, (uint32_t)i, c3, R.key0, R.key1);
            rj = (int32_t)n + (o.x < t ? 1 : 0);
            r[j] = rj;
        }
        loc[q] = sum;
        sum += rj;
    }
    int32_t tot;
    const int32_t pre = block_exscan<int32_t, CH_THREADS>(sum, lds, &tot);
    int32_t *C = R.C[it.pop];
#pragma unroll
    for (int q = 0; q < CH_PER; ++q)
        if (jb + q < Rp) C[jb + q] = pre + loc[q];
    if (threadIdx.x == 0) R.tot32[it.pop][it.chunk] = tot;
}

// Multinomial draws: draw d picks the parent j with P_j <= t < P_j + X_j,
// t = floor(v S_X / 2^64), v = o0 | o1 << 32 of Philox(seed; d, 0, i,
// TAG_MN << 28 | pop << 24); P_j = base64[chunk] + chunk-local prefix.
// `split` workgroups per chunk item (1 or CH_PER): a run that fits one
// chunk is drawn by the first of them alone; in larger runs each takes
// CH_PER / split rounds of CH_THREADS draws, one per thread and round (the
// searches are chains of dependent loads at scattered addresses, so with
// split = CH_PER they are spread over as many compute units as possible).
__global__ void __launch_bounds__(CH_THREADS) k_mn_draws(const ChunkItem *items, const RunInfo *runs,
                                                          const PopState *st, int split)
{
    const int part = blockIdx.x % split;
    const ChunkItem it = items[blockIdx.x / split];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S) || R.resampling != PA_MULTINOMIAL) return;
    const int d0 = it.chunk * CH;
    if (d0 >= R.R) return;
    const int Rp = S.Rprev;
    const uint64_t SX = S.SX;
    const uint64_t *P = R.P[it.pop];
    const uint64_t *B = R.base64[it.pop];
    const uint32_t c3 = (TAG_MN << 28) | ((uint32_t)it.pop << 24);
    int32_t *r = R.r[it.pop];
    __shared__ uint64_t sP[CH];   // one chunk's prefix, or the chunk bases
    __shared__ int32_t sr[CH];
    if (R.R <= CH && Rp <= CH) {
        // the whole run in this workgroup: prefix and counts in LDS, the
        // counts are written out once (no global atomics)
        if (part != 0) return;
        for (int j = threadIdx.x; j < Rp; j += CH_THREADS) {
            sP[j] = P[j];     // one chunk: base64[0] = 0
            sr[j] = 0;
        }
        __syncthreads();
        for (int q = 0; q < CH_PER; ++q) {
            const int d = threadIdx.x + q * CH_THREADS;
            if (d >= R.R) break;
            const u32x4 o = philox10((uint32_t)d, 0, (uint32_t)S.i, c3, R.key0, R.key1);
            const uint64_t v = (uint64_t)o.x | ((uint64_t)o.y << 32);
            const uint64_t t = umul64hi(v, SX);
            int lo = 0, hi = Rp - 1;
            while (lo < hi) {
                const int mid = lo + ((hi - lo + 1) >> 1);
                if (sP[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            atomicAdd(&sr[lo], 1);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < Rp; j += CH_THREADS) r[j] = sr[j];
        return;
    }
    // largest j with P_j <= t in two levels: the last chunk whose base is
    // <= t (chunk bases staged in LDS), then inside that chunk
    const int nch = (Rp + CH - 1) / CH;
    uint64_t *sB = sP;
    const bool staged = nch <= CH;
    if (staged)
        for (int k = threadIdx.x; k < nch; k += CH_THREADS) sB[k] = B[k];
    __syncthreads();
    // Fixed power-of-two steps: the largest index whose key is <= t,
    // starting from index 0, whose key is 0.
    for (int q = part; q < CH_PER; q += split) {
        const int d = d0 + q * CH_THREADS + (int)threadIdx.x;
        if (d >= R.R) break;
        const u32x4 o = philox10((uint32_t)d, 0, (uint32_t)S.i, c3, R.key0, R.key1);
        const uint64_t v = (uint64_t)o.x | ((uint64_t)o.y << 32);
        uint64_t t = umul64hi(v, SX);
        int k = 0;
        for (int step = nch > 1 ? 1 << (31 - __builtin_clz(nch - 1)) : 0; step > 0; step >>= 1) {
            const int m = k + step;
            if (m < nch && (staged ? sB[m] : B[m]) <= t) k = m;
        }
        t -= staged ? sB[k] : B[k];
        const uint64_t *Pk = P + (size_t)k * CH;
        const int nk = min(CH, Rp - k * CH);
        int lo = 0;
        for (int step = CH / 2; step > 0; step >>= 1) {
            const int m = lo + step;
            if (m < nk && Pk[m] <= t) lo = m;
        }
        atomicAdd(&r[k * CH + lo], 1);
    }
}

// Multinomial: chunk-local exclusive prefix of the counts r.
__global__ void __launch_bounds__(CH_THREADS) k_cnt_scan_chunk(const ChunkItem *items, const RunInfo *runs,
                                                                const PopState *st)
{
    __shared__ int32_t lds[CH_THREADS / 64 + 1];
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S) || R.resampling != PA_MULTINOMIAL) return;
    const int Rp = S.Rprev;
    const int j0 = it.chunk * CH;
    if (j0 >= Rp) return;
    const int jb = j0 + threadIdx.x * CH_PER;
    const int32_t *r = R.r[it.pop];
    int32_t loc[CH_PER];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        loc[q] = sum;
        if (jb + q < Rp) sum += r[jb + q];
    }
    int32_t tot;
    const int32_t pre = block_exscan<int32_t, CH_THREADS>(sum, lds, &tot);
    int32_t *C = R.C[it.pop];
#pragma unroll
    for (int q = 0; q < CH_PER; ++q)
        if (jb + q < Rp) C[jb + q] = pre + loc[q];
    if (threadIdx.x == 0) R.tot32[it.pop][it.chunk] = tot;
}

__device__ __forceinline__ pa_obs &obs_at(const RunInfo &R, int i, int pop)
{
    return R.obs[(size_t)i * R.obs_stride + R.obs_off + pop];
}

__device__ void freeze_run(const RunInfo &R, PopState &S, int pop, int i, int32_t status)
{
    for (int k = i + threadIdx.x; k < R.K; k += blockDim.x) {
        pa_obs o = {};
        o.status = status;
        obs_at(R, k, pop) = o;
    }
    if (threadIdx.x == 0) {
        S.status = status;
        S.moved = 0;
    }
}

// Chunk bases of the count prefix, R_i = sum r_j; capacity and empty-
// population checks (the run is frozen with that status); otherwise the
// new population becomes current: the copy reads buffer src, writes cur.
__global__ void k_cnt_finish(const RunInfo *runs, PopState *st)
{
    __shared__ int64_t lds64[257];
    const int run = blockIdx.x, pop = blockIdx.y;
    const RunInfo &R = runs[run];
    if (pop >= R.npop) return;
    PopState &S = st[run * MAX_POP + pop];
    if (!pop_active(S)) return;
    const int Rp = S.Rprev;
    const int nch = (Rp + CH - 1) / CH;
    int64_t carry = 0;
    for (int base = 0; base < nch; base += 256) {
        const int c = base + threadIdx.x;
        const int64_t v = c < nch ? R.tot32[pop][c] : 0;
        int64_t tot;
        const int64_t pre = block_exscan<int64_t, 256>(v, lds64, &tot);
        if (c < nch) R.base32[pop][c] = (int32_t)(carry + pre);
        carry += tot;
    }
    __syncthreads();
    if (carry > R.R_cap) {
        freeze_run(R, S, pop, S.i, PA_ERR_CAPACITY);
        return;
    }
    if (carry == 0) {
        freeze_run(R, S, pop, S.i, PA_ERR_NUMERIC);
        return;
    }
    if (threadIdx.x == 0) {
        S.src = S.cur;
        S.cur = S.cur ^ 1;
        S.Rcur = (int32_t)carry;
    }
}

// Parent of every child slot: parent j's r_j children occupy the slots
// C_j .. C_j + r_j - 1 (C_j = base32[chunk] + chunk-local prefix), so each
// parent writes its own.  A lane writes the first few; the slots of larger
// families are written by the whole wavefront, one family at a time.
constexpr int PARENT_LANE_MAX = 4;

__global__ void __launch_bounds__(CH_THREADS) k_parent(const ChunkItem *items, const RunInfo *runs,
                                                        const PopState *st)
{
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rp = S.Rprev;
    const int j0 = it.chunk * CH;
    if (j0 >= Rp) return;
    const int lane = threadIdx.x & 63;
    const int32_t *C = R.C[it.pop];
    const int32_t *r = R.r[it.pop];
    const int32_t base = R.base32[it.pop][it.chunk];
    int32_t *par = R.parent[it.pop];
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        const int j = j0 + q * CH_THREADS + (int)threadIdx.x;
        int rj = 0, cj = 0;
        if (j < Rp) {
            rj = r[j];
            cj = base + C[j];
        }
        const int mine = min(rj, PARENT_LANE_MAX);
        for (int m = 0; m < mine; ++m) par[cj + m] = j;
        uint64_t big = __ballot(rj > PARENT_LANE_MAX);
        while (big) {
            const int src = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            const int bj = __builtin_amdgcn_readlane(j, src), bc = __builtin_amdgcn_readlane(cj, src),
                      br = __builtin_amdgcn_readlane(rj, src);
            for (int m = PARENT_LANE_MAX + lane; m < br; m += 64) par[bc + m] = bj;
        }
    }
}

// Copy of spins, energies and family labels into the child slots.  One
// wavefront per 64 children (one replica group) and 64 sites at a time.
// MSC: the children's parents lie in a few consecutive source groups; each
// source block (64 sites x 64 replicas) is transposed so that a lane holds
// one replica's 64 sites, every child pulls its parent's row from the lane
// that holds it, and the child block is transposed back and stored
// (falls back to a per-site bit gather when the parents span many groups).
// int8: lane = child, one byte per site.
constexpr int COPY_MAX_SRC = 4;

template <int REPR>
__device__ __forceinline__ void copy_group(const RunInfo &R, const PopState &S, int pop, int G, int sub, int wpg)
{
    const int Rc = S.Rcur;
    const int lane = threadIdx.x & 63;
    const int c = G * 64 + lane;
    const bool valid = c < Rc;
    const int clast = min(Rc, G * 64 + 64) - 1;
    const int p = R.parent[pop][valid ? c : clast];
    const int N = R.N;
    if (REPR == PA_MSC64) {
        const uint64_t *src = (const uint64_t *)R.spins[pop][S.src];
        uint64_t *dst = (uint64_t *)R.spins[pop][S.cur] + (size_t)G * N;
        // parents ascend with the children: the first and last lanes bound them
        const int g_lo = __builtin_amdgcn_readlane(p, 0) >> 6;
        const int g_hi = __builtin_amdgcn_readlane(p, 63) >> 6;
        if (g_hi - g_lo < COPY_MAX_SRC) {
            const int nsrc = g_hi - g_lo + 1;   // uniform over the wavefront
            // two 64-site blocks per step: their source loads are issued together
            for (int n0 = sub * 64; n0 < N; n0 += 2 * wpg * 64) {
                const int na = n0 + lane, nb = n0 + wpg * 64 + lane;
                uint64_t xa[COPY_MAX_SRC], xb[COPY_MAX_SRC];
#pragma unroll
                for (int q = 0; q < COPY_MAX_SRC; ++q) {
                    const size_t gofs = (size_t)(g_lo + q) * N;
                    xa[q] = (q < nsrc && na < N) ? src[gofs + na] : 0ull;
                    xb[q] = (q < nsrc && nb < N) ? src[gofs + nb] : 0ull;
                }
                uint64_t rowa = 0, rowb = 0;
#pragma unroll
                for (int q = 0; q < COPY_MAX_SRC; ++q) {
                    if (q < nsrc) {
                        const uint64_t va = __shfl(transpose64(xa[q]), p & 63, 64);
                        const uint64_t vb = __shfl(transpose64(xb[q]), p & 63, 64);
                        if ((p >> 6) == g_lo + q) {
                            rowa = va;
                            rowb = vb;
                        }
                    }
                }
                if (!valid) rowa = rowb = 0;
                const uint64_t outa = transpose64(rowa), outb = transpose64(rowb);
                if (na < N) dst[na] = outa;
                if (nb < N) dst[nb] = outb;
            }
        } else {
            const uint64_t *ps = src + (size_t)(p >> 6) * N;
            const int pb = p & 63;
            for (int nb = sub * 64; nb < N; nb += wpg * 64) {
                uint64_t mine = 0;
                const int cnt = min(64, N - nb);
                for (int k = 0; k < cnt; ++k) {
                    const int bit = valid ? (int)((ps[nb + k] >> pb) & 1u) : 0;
                    const uint64_t m = __ballot(bit);
                    if (lane == k) mine = m;
                }
                if (lane < cnt) dst[nb + lane] = mine;
            }
        }
    } else if ((__builtin_amdgcn_readlane(p, 63) >> 6) - (__builtin_amdgcn_readlane(p, 0) >> 6) < 2) {
        // the parents lie in at most two source groups: each lane packs the
        // 64 spin bytes of one site of each source group into a word (16-byte
        // loads), the words go through the bit-packed copy above, and the
        // child word is unpacked into 64 canonical bytes (16-byte stores)
        const uint8_t *srcb = R.spins[pop][S.src];
        uint8_t *dstb = R.spins[pop][S.cur] + (size_t)G * N * 64;
        const int g_lo = __builtin_amdgcn_readlane(p, 0) >> 6;
        const int nsrc = (__builtin_amdgcn_readlane(p, 63) >> 6) - g_lo + 1;   // 1 or 2, uniform
        for (int n0 = sub * 64; n0 < N; n0 += 2 * wpg * 64) {
            uint4 v[2][2][4];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int n = min(n0 + b * wpg * 64 + lane, N - 1);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint4 *s4 = (const uint4 *)(srcb + ((size_t)(g_lo + min(q, nsrc - 1)) * N + n) * 64);
#pragma unroll
                    for (int k = 0; k < 4; ++k) v[b][q][k] = s4[k];
                }
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                uint64_t row = 0;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (q < nsrc) {
                        const uint64_t t = __shfl(transpose64(pack64(v[b][q])), p & 63, 64);
                        if ((p >> 6) == g_lo + q) row = t;
                    }
                }
                if (!valid) row = 0;   // slots past the population hold +1 spins
                const uint64_t out = transpose64(row);
                const int n = n0 + b * wpg * 64 + lane;
                if (n0 + b * wpg * 64 < N && n < N) {
                    uint4 *d4 = (uint4 *)(dstb + (size_t)n * 64);
#pragma unroll
                    for (int k = 0; k < 4; ++k) d4[k] = spins16((uint32_t)(out >> (16 * k)) & 0xFFFFu);
                }
            }
        }
    } else {
        const uint8_t *src = R.spins[pop][S.src] + (size_t)(p >> 6) * N * 64 + (p & 63);
        uint8_t *dst = R.spins[pop][S.cur] + (size_t)G * N * 64 + lane;
        // eight sites per step, all loads issued before the stores (the
        // buffers differ, but the compiler cannot know it)
        constexpr int U = 8;
        for (int n0 = sub; n0 < N; n0 += U * wpg) {
            uint8_t v[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int n = n0 + q * wpg;
                v[q] = (valid && n < N) ? src[(size_t)n * 64] : (uint8_t)1;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int n = n0 + q * wpg;
                if (n < N) dst[(size_t)n * 64] = v[q];
            }
        }
    }
    if (sub == 0 && valid) {
        R.E[pop][S.cur][c] = R.E[pop][S.src][p];
        R.fam[pop][S.cur][c] = R.fam[pop][S.src][p];
    }
}

// Workgroup b of a launch runs on XCD b mod 8 (round-robin dispatch, one L2
// per XCD).  The item taken by b gives every XCD a contiguous range of
// items, so neighbouring items share their XCD's L2.  A bijection of
// [0, n) for any n.
__device__ __forceinline__ int xcd_item(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Workgroups of MEAS_WAVES wavefronts over the measure items: each group
// gets meas_waves_per_group(N) wavefronts, which split its sites.  The
// children of neighbouring groups have parents in shared source groups, so
// neighbouring items run on one XCD.
// split workgroups share an item: workgroup h of it takes the h-th share of
// each group's 64-site blocks (more wavefronts in flight for large lattices,
// each with a shorter chain of loads and transposes).
template <int REPR>
__global__ void __launch_bounds__(MEAS_THREADS) k_copy(const SweepItem *items, const RunInfo *runs,
                                                       const PopState *st, int split)
{
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const SweepItem it = items[b / split];
    const int h = b - (b / split) * split;
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int wpg = meas_waves_per_group(R.N);
    const int wv = wave_id();
    const int k = wv / wpg, sub = wv - k * wpg;
    const int G = it.group0 + k;
    if (k >= it.ngroups || G * 64 >= S.Rcur) return;
    copy_group<REPR>(R, S, it.pop, G, h * wpg + sub, split * wpg);
}

// ------------------------------------------------------------- step (iv)

// The sweep kernels' exact work counters: one set of atomics per
// wavefront, into a slot chosen by workgroup and wavefront.
__device__ __forceinline__ void flush_stats(unsigned long long *stats, uint64_t words, uint32_t calls,
                                            uint64_t flips)
{
    const unsigned long long w = wave_sum<unsigned long long>(words);
    const unsigned long long c = wave_sum<unsigned long long>(calls);
    const unsigned long long f = wave_sum<unsigned long long>(flips);
    if ((threadIdx.x & 63) == 0) {
        const unsigned slot = (blockIdx.x * 16u + (threadIdx.x >> 6)) % STAT_SLOTS;
        unsigned long long *p = stats + (size_t)slot * NSTAT;
        atomicAdd(&p[ST_WORDS], w);
        atomicAdd(&p[ST_CALLS], c);
        atomicAdd(&p[ST_FLIPS], f);
    }
}

__device__ __forceinline__ uint64_t jmask(uint8_t b, int bit) { return ((b >> bit) & 1u) ? ~0ull : 0ull; }

// Plain path: one colour of one run per launch, int8 spins ([group][site][64
// replicas] bytes).  A workgroup takes `rows` lattice rows of one replica
// group, plus one halo row on each side unless it holds the whole lattice.
// All of its 16-byte chunks are loaded first (consecutive lanes take
// consecutive chunks, so the loads coalesce and are all in flight at once),
// their sign bits are packed into an LDS bit-lattice (one 64-bit word per
// site), the colour's sites are updated from the packed words, and the
// chunks that change are rebuilt from their signs and stored.
constexpr int I8_CMAX = 12;   // 16-byte chunks held per thread

// Rows per workgroup of the plain sweep: the whole lattice if its chunks fit
// in `threads` threads' registers, else the largest divisor T of L whose
// T + 2 rows (with halos) fit.
constexpr int int8_rows_for(int L, int threads)
{
    const int cap = threads * I8_CMAX;
    if (L * L * 4 <= cap) return L;
    int best = 1;
    for (int T = 1; T < L; ++T)
        if (L % T == 0 && (T + 2) * L * 4 <= cap) best = T;
    return best;
}

template <int LT, int THREADS>
__device__ __forceinline__ void sweep_int8_tile(const RunInfo &R, const PopState &S, int pop, int g, int tile,
                                                int s, int colour, int T, uint64_t *sm, unsigned long long *stats)
{
    const int L = LT ? LT : R.L;
    const int N = L * L, half = L >> 1;
    const int Rc = S.Rcur;
    const int y0 = tile * T;
    const int rows = min(T, L - y0);
    const int halo = rows == L ? 0 : 1;
    const int nrow = rows + 2 * halo;
    constexpr int nthr = THREADS;
    const int tid = threadIdx.x;
    uint64_t *packed = sm;                              // [nrow][L]
    uint64_t *fm = sm + (size_t)nrow * L;               // [rows][half]
    uint16_t *pk16 = (uint16_t *)packed;
    uint8_t *base = R.spins[pop][S.cur] + (size_t)g * N * 64;
    const int i = S.i;
    const Thresholds Th = thresholds_of(R.tabT, i);
    const uint32_t key0 = R.key0, key1 = R.key1;
    const uint8_t *jbits = R.jbits;
    const int chunks = nrow * L * 4;
    uint4 reg[I8_CMAX];
    // byte offset of chunk c inside the group's N * 64 bytes
    auto off_of = [&](int c) {
        const int site = c >> 2, part = c & 3;
        const int rr = site / L, x = site - rr * L;
        int y = y0 - halo + rr;
        y = y < 0 ? y + L : (y >= L ? y - L : y);
        return (uint32_t)(y * L + x) * 64u + (uint32_t)part * 16u;
    };
    // Every load is issued before the first use, with no branch around any
    // of them (a branch would make each load wait for its registers at the
    // join): lanes past the last chunk load that chunk again, in bounds.  For
    // a lattice size known here the tile and so the number of loads per
    // thread are compile-time constants.
    constexpr int QN = LT ? (((LT == int8_rows_for(LT, THREADS) ? LT : int8_rows_for(LT, THREADS) + 2) * LT * 4 +
                              THREADS - 1) / THREADS)
                          : I8_CMAX;
    static_assert(QN <= I8_CMAX, "tile chunks exceed the registers held per thread");
#pragma unroll
    for (int q = 0; q < QN; ++q)
        reg[q] = *(const uint4 *)(base + off_of(min(tid + q * nthr, chunks - 1)));
#pragma unroll
    for (int q = 0; q < I8_CMAX; ++q) {
        const int c = tid + q * nthr;
        if (c < chunks) pk16[c] = (uint16_t)signs16(reg[q]);
    }
    __syncthreads();
    const uint32_t c3 = (TAG_SWEEP << 28) | ((uint32_t)pop << 24) | (uint32_t)s;
    const uint64_t valid = (Rc - g * 64 >= 64) ? ~0ull : ((1ull << (Rc - g * 64)) - 1);
    const uint32_t lanes = (uint32_t)__popcll(valid);
    uint32_t nwords = 0, ncalls = 0;
    for (int idx = tid; idx < rows * half; idx += nthr) {
        const int yy = idx / half, m = idx - yy * half;
        const int y = y0 + yy;
        const int x = 2 * m + ((y + colour) & 1);
        const int n = y * L + x;
        const int xr = x + 1 == L ? 0 : x + 1, xl = x == 0 ? L - 1 : x - 1;
        const int yu = y == 0 ? L - 1 : y - 1;
        const int rc = yy + halo;
        const int rd = halo ? rc + 1 : (rc + 1 == L ? 0 : rc + 1);
        const int ru = halo ? rc - 1 : (rc == 0 ? L - 1 : rc - 1);
        const uint64_t w = packed[rc * L + x];
        const uint8_t jn = jbits[n];
        fm[idx] = flip_mask(w, packed[rc * L + xr], packed[rc * L + xl], packed[rd * L + x], packed[ru * L + x],
                            jmask(jn, 0), jmask(jbits[y * L + xl], 0), jmask(jn, 1), jmask(jbits[yu * L + x], 1),
                            Th, valid, (uint32_t)n, (uint32_t)g, (uint32_t)i, c3, key0, key1, ncalls);
        ++nwords;
    }
    __syncthreads();
    // Store: one 16-byte chunk of a colour site per lane step (idx as in the
    // update loop).  Spins are the canonical bytes +1 = 0x01, -1 = 0xFF, so a
    // chunk is rebuilt from its packed sign bits and flips; the registers that
    // held the loads are free during the update.
    for (int k = tid; k < rows * half * 4; k += nthr) {
        const int idx = k >> 2, part = k & 3;
        const uint32_t f = (uint32_t)(fm[idx] >> (16 * part)) & 0xFFFFu;
        if (f) {
            const int yy = idx / half, m = idx - yy * half;
            const int y = y0 + yy;
            const int x = 2 * m + ((y + colour) & 1);
            const uint32_t b = f ^ (uint32_t)pk16[((yy + halo) * L + x) * 4 + part];
            const uint4 v = spins16(b);
            *(uint4 *)(base + (uint32_t)(y * L + x) * 64u + (uint32_t)part * 16u) = v;
        }
    }
    flush_stats(stats, nwords, ncalls, nwords * lanes);
}

// THREADS: the workgroup size it is launched with (256, or 1024 for very
// large lattices); the bound lets the 256-thread form keep its chunks and
// the Philox state in registers instead of spilling them to scratch.
template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_sweep_int8(const RunInfo *runs, const PopState *st, int run, int pop,
                                                        int s, int colour, int T, int ntiles,
                                                        unsigned long long *stats)
{
    extern __shared__ uint64_t sm[];
    const RunInfo &R = runs[run];
    const PopState &S = st[run * MAX_POP + pop];
    if (!pop_active(S)) return;
    const int g = blockIdx.x / ntiles, tile = blockIdx.x - g * ntiles;
    if (g * 64 >= S.Rcur) return;
    switch (R.L) {
    case 8: sweep_int8_tile<8, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    case 16: sweep_int8_tile<16, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    case 24: sweep_int8_tile<24, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    case 32: sweep_int8_tile<32, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    case 48: sweep_int8_tile<48, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    case 64: sweep_int8_tile<64, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    default: sweep_int8_tile<0, THREADS>(R, S, pop, g, tile, s, colour, T, sm, stats); break;
    }
}

// Batched path: every (run, pop, block of G replica groups) item of the
// context in one launch.  The G lattices (colour-split, so a colour's sites
// are contiguous) and the couplings stay in LDS for all theta sweeps.
//
// Draw scheduling.  A site needs as many Philox calls as its slowest
// undecided replica (about 3-4 on average, up to 16).  Each wavefront owns a
// contiguous range of a colour's sites and works in rounds with one call
// index per round, uniform across the wavefront:
//  - dense rounds: chunks of 64 sites are classified (always flip / dE = +4 /
//    dE = +8) and make calls 0 .. dense-1 in lockstep; nearly every site
//    needs that many, so few lanes idle;
//  - sparse rounds: the sites still undecided are kept in a wave-private LDS
//    list.  For lattices of at most 4096 sites the list is a queue (a ring
//    of at most MSC_QUEUE_SLOTS entries in the kernels compiled for one
//    size) whose entries carry their next call index, and every round takes
//    the next 64 entries whatever call each is at (stream_rounds,
//    stream_tail); otherwise the list is compacted in place after every
//    call index (sweep_sparse_wave), or pooled over the workgroup
//    (sweep_sparse_pooled).  Either way each round's calls run on full
//    wavefronts until the last entries.
// Every site's result is still the plain most-significant-first comparison
// of its own bit planes; only the order of the work changes.

// Lanes of the wavefront where p holds.  Unlike __ballot(int), the
// predicate stays a lane mask: a condition combined from several compares
// is not turned into an integer and compared again.
__device__ __forceinline__ uint64_t wave_ballot(bool p)
{
    return __builtin_amdgcn_ballot_w64(p);
}

// Flips the accepted replicas of a lattice word in LDS with one atomic XOR
// that returns nothing: no read into registers, no wait, and no test for an
// empty mask (XOR with zero changes nothing).  The words of one round are
// distinct sites, and a wavefront's LDS operations complete in order.
__device__ __forceinline__ void flip_word(uint64_t *w, uint64_t acc)
{
    __hip_atomic_fetch_xor(w, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// b plus the number of lanes below this one whose bit is set in the
// wavefront mask m (two mbcnt instructions).
__device__ __forceinline__ int rank_below(uint64_t m, int b)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)b));
}

// x mod m for 0 <= x < 2m: an unsigned minimum instead of a compare and a
// select.
__device__ __forceinline__ int wrap_once(int x, int m)
{
    return (int)min((uint32_t)x, (uint32_t)x - (uint32_t)m);
}

// A list entry's undecided lanes of the two classes (dE = +4, dE = +8), kept
// side by side so that one LDS address serves both.  Reads are one 16-byte
// access (ds_read_b128).  Writes go out as two 8-byte halves of one
// instruction (ds_write2_b64): with 16-byte writes the wavefronts waited
// longer for LDS issue and the sweep was slower.
struct alignas(16) UndPair {
    uint64_t u4, u8;
};

__device__ __forceinline__ void und_load(const UndPair *p, uint64_t &u4, uint64_t &u8)
{
    const UndPair v = *p;
    u4 = v.u4;
    u8 = v.u8;
}

__device__ __forceinline__ void und_store(UndPair *p, uint64_t u4, uint64_t u8)
{
    uint64_t *w = (uint64_t *)(void *)p;   // 8-byte alignment: two 8-byte halves
    w[0] = u4;
    w[1] = u8;
}

// Sparse rounds of one wavefront over its own compacted list of `cnt`
// undecided sites (entries: lanes of each class, LDS word << 16 | site):
// call c for every entry, survivors compacted in place; once one pass holds
// every remaining entry it runs all their remaining calls without writing
// the list back.
__device__ __forceinline__ void sweep_sparse_wave(uint64_t *lat, UndPair *eu, uint32_t *en, int cnt,
                                                  int c_first, int N, int group0, const Thresholds &Th, uint32_t i,
                                                  uint32_t c3, uint32_t key0, uint32_t key1, uint32_t &wcalls)
{
    const int lane = threadIdx.x & 63;
    for (int c = c_first; c < 16 && cnt > 0; ++c) {
        if (cnt <= 64) {
            uint64_t und4 = 0, und8 = 0, acc = 0;
            int addr = 0;
            uint32_t n = 0, g = 0;
            if (lane < cnt) {
                und_load(&eu[lane], und4, und8);
                const uint32_t pk = en[lane];
                addr = (int)(pk >> 16);
                n = pk & 0xFFFFu;
                g = (uint32_t)(group0 + addr / N);
            }
            for (; c < 16; ++c) {
                const uint64_t live = wave_ballot((und4 | und8) != 0);
                if (live == 0) break;
                wcalls += (uint32_t)__popcll(live);
                if ((und4 | und8) != 0) draw_call((uint32_t)c, Th.t4, Th.t8, und4, und8, acc, n, g, i, c3, key0, key1);
            }
            flip_word(&lat[addr], acc);
            return;
        }
        int wcnt = 0;
        for (int e0 = 0; e0 < cnt; e0 += 64) {
            const int e = e0 + lane;
            uint64_t und4 = 0, und8 = 0, acc = 0;
            uint32_t pk = 0;
            wcalls += (uint32_t)min(64, cnt - e0);
            if (e < cnt) {
                und_load(&eu[e], und4, und8);
                pk = en[e];
                const int addr = (int)(pk >> 16);
                const uint32_t g = (uint32_t)(group0 + addr / N);
                draw_call((uint32_t)c, Th.t4, Th.t8, und4, und8, acc, pk & 0xFFFFu, g, i, c3, key0, key1);
                flip_word(&lat[addr], acc);
            }
            const uint64_t need = wave_ballot((und4 | und8) != 0);
            if ((und4 | und8) != 0) {
                const int slot = rank_below(need, wcnt);
                und_store(&eu[slot], und4, und8);
                en[slot] = pk;
            }
            wcnt += __popcll(need);
        }
        cnt = wcnt;
    }
}

// Sparse rounds of one wavefront as a stream (lattices of at most 4096
// sites): its undecided sites form a queue in a ring of `cap` slots (an
// entry is LDS word << 16 | its next call << 12 | site).  Every round takes
// the next 64 entries, whatever call each is at, makes that call, and
// appends the sites still undecided at the tail with their next call, so
// rounds stay full until fewer than 64 entries remain; those then run all
// their remaining calls without being written back (stream_tail).  The
// dense chunks append to the same ring; when it is smaller than the
// wavefront's range, full rounds run between chunks whenever it holds more
// than 64 entries, so the next chunk's entries always fit.  Each site keeps
// the plain most-significant-first comparison of its own bit planes; only
// the order of the work changes.  tmask[c] holds T's bits at the planes of
// call c (call_masks); with ONE_GROUP (the workgroup holds one replica
// group) every entry's group is group0, a uniform value.
struct Ring {
    int hs, ts, left;   // slot of the head, slot of the tail, entries
};

// Full rounds while the ring holds more than `limit` (>= 64) entries.
template <bool ONE_GROUP>
__device__ __forceinline__ void stream_rounds(Ring &q, int limit, uint64_t *lat, UndPair *eu,
                                              uint32_t *en, int cap, int N, int group0, const uint4 *tmask,
                                              uint32_t i, uint32_t c3, uint32_t key0, uint32_t key1,
                                              uint32_t &wcalls)
{
    const int lane = threadIdx.x & 63;
    auto group_of = [&](int addr) { return (uint32_t)(ONE_GROUP ? group0 : group0 + addr / N); };
    int left = q.left, hs = q.hs, ts = q.ts;
    while (left > limit) {
        const int slot = wrap_once(hs + lane, cap);
        uint64_t und4, und8, acc = 0;
        und_load(&eu[slot], und4, und8);
        const uint32_t pk = en[slot];
        const int addr = (int)(pk >> 16);
        const uint32_t c = (pk >> 12) & 15u;
        draw_call_masks(c, tmask[c], und4, und8, acc, pk & 0xFFFu, group_of(addr), i, c3, key0, key1);
        wcalls += 64;
        flip_word(&lat[addr], acc);
        const bool more = (und4 | und8) != 0 && c < 15u;
        // the two compares' masks, combined on the scalar unit
        const uint64_t need = wave_ballot((und4 | und8) != 0) & wave_ballot(c < 15u);
        if (more) {
            const int out = wrap_once(rank_below(need, ts), cap);
            und_store(&eu[out], und4, und8);
            en[out] = (pk & 0xFFFF0FFFu) | ((c + 1u) << 12);
        }
        const int nn = __popcll(need);
        ts += nn;
        if (ts >= cap) ts -= cap;
        hs += 64;
        if (hs >= cap) hs -= cap;
        left += nn - 64;
    }
    q.left = left;
    q.hs = hs;
    q.ts = ts;
}

// The last (at most 64) entries: each lane runs all the remaining calls of
// its own entry.
template <bool ONE_GROUP>
__device__ __forceinline__ void stream_tail(const Ring &q, uint64_t *lat, const UndPair *eu,
                                            const uint32_t *en, int cap, int N, int group0, const uint4 *tmask,
                                            uint32_t i, uint32_t c3, uint32_t key0, uint32_t key1,
                                            uint32_t &wcalls)
{
    const int lane = threadIdx.x & 63;
    uint64_t und4 = 0, und8 = 0, acc = 0;
    int addr = 0;
    uint32_t n = 0, c = 16;
    if (lane < q.left) {
        const int slot = wrap_once(q.hs + lane, cap);
        und_load(&eu[slot], und4, und8);
        const uint32_t pk = en[slot];
        addr = (int)(pk >> 16);
        c = (pk >> 12) & 15u;
        n = pk & 0xFFFu;
    }
    const uint32_t g = (uint32_t)(ONE_GROUP ? group0 : group0 + addr / N);
    for (;;) {
        const bool live = (und4 | und8) != 0 && c < 16u;
        const uint64_t lv = wave_ballot((und4 | und8) != 0) & wave_ballot(c < 16u);
        if (lv == 0) break;
        wcalls += (uint32_t)__popcll(lv);
        if (live) {
            draw_call_masks(c, tmask[c], und4, und8, acc, n, g, i, c3, key0, key1);
            ++c;
        }
    }
    flip_word(&lat[addr], acc);
}

// Sparse rounds over one list shared by the workgroup (ctl[h & 1] entries,
// appended by every wavefront in the dense rounds): each round takes the
// list in passes of one wavefront-load per wavefront; after a pass the
// wavefronts' survivor counts (ctl[2 + 16 par + w], alternating buffers)
// give every survivor its place in the compacted list, which always lies
// before the entries of later passes, so the list is compacted in place.
// When at most two wavefront-loads remain, two wavefronts (one if the
// workgroup has only one) run all their remaining calls without writing the
// list back.
__device__ __forceinline__ void sweep_sparse_pooled(uint64_t *lat, UndPair *eu, uint32_t *en,
                                                    int *ctl, int h, int c_first, int N, int group0,
                                                    const Thresholds &Th, uint32_t i, uint32_t c3, uint32_t key0,
                                                    uint32_t key1, uint32_t &wcalls)
{
    const int lane = threadIdx.x & 63, wv = wave_id(), nw = blockDim.x >> 6;
    const int tailw = min(2, nw);   // wavefronts that finish the last entries
    __syncthreads();   // every wavefront's appends are in the list
    int cnt = ctl[h & 1];
    int par = 0;
    for (int c = c_first; c < 16 && cnt > 0; ++c) {
        if (cnt <= 64 * tailw) {
            if (wv < tailw) {
                const int e = wv * 64 + lane;
                uint64_t und4 = 0, und8 = 0, acc = 0;
                int addr = 0;
                uint32_t n = 0, g = 0;
                if (e < cnt) {
                    und_load(&eu[e], und4, und8);
                    const uint32_t pk = en[e];
                    addr = (int)(pk >> 16);
                    n = pk & 0xFFFFu;
                    g = (uint32_t)(group0 + addr / N);
                }
                for (; c < 16; ++c) {
                    const uint64_t live = wave_ballot((und4 | und8) != 0);
                    if (live == 0) break;
                    wcalls += (uint32_t)__popcll(live);
                    if ((und4 | und8) != 0)
                        draw_call((uint32_t)c, Th.t4, Th.t8, und4, und8, acc, n, g, i, c3, key0, key1);
                }
                flip_word(&lat[addr], acc);
            }
            return;
        }
        int out = 0;
        for (int s0 = 0; s0 < cnt; s0 += 64 * nw) {
            const int e = s0 + wv * 64 + lane;
            uint64_t und4 = 0, und8 = 0, acc = 0;
            uint32_t pk = 0;
            wcalls += (uint32_t)max(0, min(64, cnt - (s0 + wv * 64)));
            if (e < cnt) {
                und_load(&eu[e], und4, und8);
                pk = en[e];
                const int addr = (int)(pk >> 16);
                const uint32_t g = (uint32_t)(group0 + addr / N);
                draw_call((uint32_t)c, Th.t4, Th.t8, und4, und8, acc, pk & 0xFFFFu, g, i, c3, key0, key1);
                flip_word(&lat[addr], acc);
            }
            const uint64_t need = wave_ballot((und4 | und8) != 0);
            int *cw = ctl + 2 + 16 * par;
            if (lane == 0) cw[wv] = __popcll(need);
            __syncthreads();
            int off = out, tot = 0;
            for (int w = 0; w < nw; ++w) {
                const int v = cw[w];
                off += w < wv ? v : 0;
                tot += v;
            }
            if ((und4 | und8) != 0) {
                const int slot = rank_below(need, off);
                und_store(&eu[slot], und4, und8);
                en[slot] = pk;
            }
            out += tot;
            par ^= 1;
        }
        __syncthreads();   // the compacted list is complete
        cnt = out;
    }
}

template <int LT, bool EA, bool RING>
__device__ __forceinline__ void sweep_item(const SweepItem &item, const RunInfo &R, const PopState &S,
                                           uint64_t *lds, int mode, unsigned long long *stats)
{
    // Everything the loops need is read into registers before the first
    // barrier: a barrier orders memory, so values left in global memory
    // would be loaded again after every one of them.
    const int L = LT ? LT : __builtin_amdgcn_readfirstlane(R.L);
    const int N = L * L, half = L >> 1, nh = N >> 1;
    const int T = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wv = wave_id(), nw = T >> 6;
    const int Rc = __builtin_amdgcn_readfirstlane(S.Rcur);
    const int group0 = __builtin_amdgcn_readfirstlane(item.group0);
    const int pop = __builtin_amdgcn_readfirstlane(item.pop);
    const int theta = __builtin_amdgcn_readfirstlane(R.theta);
    // this item's sweeps: a chunk of them (boundaries chosen by the plan,
    // expand_sweep_chunks), or all theta
    const int nchunk = max(1, __builtin_amdgcn_readfirstlane(item.nchunk));
    const int chunk = __builtin_amdgcn_readfirstlane(item.chunk);
    int s_begin = 0, s_end = theta;
    if (nchunk == 2) {
        const int cut = min(max(__builtin_amdgcn_readfirstlane(item.cut), 0), theta);
        s_begin = chunk ? cut : 0;
        s_end = chunk ? theta : cut;
    } else if (nchunk > 2) {
        const int sq = theta / nchunk, sr = theta - sq * nchunk;
        s_begin = chunk * sq + min(chunk, sr);
        s_end = s_begin + sq + (chunk < sr ? 1 : 0);
    }
    const uint32_t key0 = __builtin_amdgcn_readfirstlane(R.key0), key1 = __builtin_amdgcn_readfirstlane(R.key1);
    const int G = min(__builtin_amdgcn_readfirstlane(item.ngroups), (Rc + 63) / 64 - group0);
    if (G <= 0) return;
    const int units = G * nh;
    const bool pool = (mode >> 8) & 1;
    const int dense = mode & 0xFF;
    // the streamed sparse rounds keep each entry's next call in its site
    // word's top bits (sites < 4096); calls 0 .. 15 only
    const bool stream = msc_streamed(N, mode);
    // one list entry per unit, or (RING: the kernels compiled for one size)
    // a ring of MSC_QUEUE_SLOTS per wavefront
    const int lmode = RING ? mode : mode | MSC_WHOLE_LISTS;   // the layout the launch sized
    const int ents = msc_list_entries(N, G, nw, lmode);
    const bool bounded = ents < units;
    uint64_t *lat = lds;                                  // [G][2][nh]
    UndPair *eu = (UndPair *)(lds + (size_t)G * N);       // [ents] undecided lanes of the two classes
    uint32_t *en = (uint32_t *)(eu + ents);               // [ents] (LDS word << 16) | site
    uint8_t *jb = (uint8_t *)(en + ents);                 // [2][nh] bond signs of each site (spin glass)
    int *ctl = (int *)(jb + (EA ? N : 0));                // pooled list counts [2], pass counts [2][16]
    uint4 *tmask = (uint4 *)(lds + msc_lds_tmask_off(N, G, EA, nw, lmode) / 8);   // [16] T's bits per call
    uint64_t *base = (uint64_t *)R.spins[pop][S.cur] + (size_t)group0 * N;
    for (int u = tid; u < G * N; u += T) {
        const int gs = u / N, n = u - gs * N;
        const int y = n / L, x = n - y * L;
        lat[(size_t)gs * N + ((x + y) & 1) * nh + y * half + (x >> 1)] = base[u];
    }
    // Colour-split neighbours of site k = y half + m (x = 2m + p, p = (y +
    // colour) & 1) in the other colour's array: k itself and kh = k - 1 or
    // k + 1 within the row (the horizontal pair), k -+ half (up, down).
    // jb holds the signs of the four bonds in that order (bit set: J = -1).
    if (EA)
        for (int v = tid; v < N; v += T) {
            const int colour = v / nh, k = v - colour * nh;
            const int y = k / half, m = k - y * half;
            const int p = (y + colour) & 1, x = 2 * m + p;
            const int xl = x == 0 ? L - 1 : x - 1, yu = y == 0 ? L - 1 : y - 1;
            const uint8_t jn = R.jbits[y * L + x];
            const uint32_t jr = jn & 1u, jd = (jn >> 1) & 1u;
            const uint32_t jl = R.jbits[y * L + xl] & 1u, ju = (R.jbits[yu * L + x] >> 1) & 1u;
            // k is the right neighbour when p = 0 and the left one when p = 1
            const uint32_t jk = p ? jl : jr, jh = p ? jr : jl;
            jb[v] = (uint8_t)(jk | (jh << 1) | (ju << 2) | (jd << 3));
        }
    const int i = __builtin_amdgcn_readfirstlane(S.i);
    const Thresholds Th = thresholds_of(R.tabT, i);
    const bool saturated = Th.all4 || Th.all8;
    if (tid < 16) tmask[tid] = call_masks(Th.t4, Th.t8, (uint32_t)tid);   // read after the next barrier
    const uint32_t c3p = (TAG_SWEEP << 28) | ((uint32_t)pop << 24);
    const int lastg = group0 + G - 1;
    const uint64_t vlast = (Rc - lastg * 64 >= 64) ? ~0ull : ((1ull << (Rc - lastg * 64)) - 1);
    const int upw = (units + nw - 1) / nw;
    const int ub = min(units, wv * upw), ue = min(units, ub + upw);
    // this wavefront's ring of streamed entries: its own range of the lists,
    // or MSC_QUEUE_SLOTS slots of its own
    const int rb = bounded ? wv * MSC_QUEUE_SLOTS : ub, rcap = bounded ? MSC_QUEUE_SLOTS : ue - ub;
    uint32_t wcalls = 0;   // Philox calls of this wavefront (uniform)
    if (tid == 0) ctl[0] = ctl[1] = 0;
    for (int s = s_begin; s < s_end; ++s) {
        const uint32_t c3 = c3p | (uint32_t)s;
        for (int colour = 0; colour < 2; ++colour) {
            const int h = 2 * s + colour;   // half-sweep index: its list count is ctl[h & 1]
            __syncthreads();
            if (tid == 0) ctl[(h + 1) & 1] = 0;   // the next half-sweep's count; last read before this barrier
            int cnt = 0;
            Ring q = {0, 0, 0};
            // dense rounds, 64 units per pass; one unit (lane) per site word
            auto chunk = [&](bool live_unit, int gs, int k, int kh, int ku, int kd, int addr, uint32_t n) {
                uint64_t und4 = 0, und8 = 0, acc = 0;
                const uint32_t g = (uint32_t)(group0 + gs);
                if (live_unit) {
                    const uint64_t *oth = lat + (size_t)gs * N + (colour ^ 1) * nh;
                    const uint64_t w = lat[addr];
                    uint64_t j0 = 0, j1 = 0, j2 = 0, j3 = 0;
                    if (EA) {
                        const uint32_t jm = jb[colour * nh + k];
                        j0 = jmask((uint8_t)jm, 0);
                        j1 = jmask((uint8_t)jm, 1);
                        j2 = jmask((uint8_t)jm, 2);
                        j3 = jmask((uint8_t)jm, 3);
                    }
                    SiteClass sc = classify<EA>(w, oth[k], oth[kh], oth[ku], oth[kd], j0, j1, j2, j3);
                    if (saturated) {   // uniform, only where a threshold is 2^32 (beta_i = 0)
                        if (Th.all4) { sc.flip |= sc.one; sc.one = 0; }
                        if (Th.all8) { sc.flip |= sc.zero; sc.zero = 0; }
                    }
                    acc = sc.flip;
                    und4 = sc.one;
                    und8 = sc.zero;
                    if (group0 + gs == lastg) {   // only its valid replicas draw
                        und4 &= vlast;
                        und8 &= vlast;
                    }
                }
                for (int c = 0; c < dense; ++c) {
                    const uint64_t live = wave_ballot((und4 | und8) != 0);
                    if (live == 0) break;
                    wcalls += (uint32_t)__popcll(live);
                    if ((und4 | und8) != 0)
                        draw_call((uint32_t)c, Th.t4, Th.t8, und4, und8, acc, n, g, (uint32_t)i, c3, key0, key1);
                }
                flip_word(&lat[addr], acc);
                const uint64_t need = wave_ballot((und4 | und8) != 0);
                int base_slot = ub + cnt;
                if (pool && need) {
                    int b0 = 0;
                    if (lane == 0) b0 = atomicAdd(&ctl[h & 1], __popcll(need));
                    base_slot = __builtin_amdgcn_readlane(b0, 0);
                }
                if ((und4 | und8) != 0) {
                    const int slot =
                        stream ? rb + wrap_once(rank_below(need, q.ts), rcap) : rank_below(need, base_slot);
                    und_store(&eu[slot], und4, und8);
                    en[slot] = ((uint32_t)addr << 16) | (stream ? (uint32_t)dense << 12 : 0u) | n;
                }
                cnt += __popcll(need);
                if (stream) {
                    q.ts += __popcll(need);
                    if (q.ts >= rcap) q.ts -= rcap;
                    q.left += __popcll(need);
                    if (RING && bounded && q.left > rcap - 64) {   // room for the next chunk's entries
                        if (G == 1)
                            stream_rounds<true>(q, rcap - 64, lat, eu + rb, en + rb, rcap, N, group0, tmask,
                                                (uint32_t)i, c3, key0, key1, wcalls);
                        else
                            stream_rounds<false>(q, rcap - 64, lat, eu + rb, en + rb, rcap, N, group0,
                                                 tmask, (uint32_t)i, c3, key0, key1, wcalls);
                    }
                }
            };
            // Strength-reduced indices: when a pass starts on a multiple of
            // 64 units, a row half (L/2 words) divides 64 an even number of
            // times and a colour's half-lattice (N/2 words) is a multiple of
            // 64, every lane keeps its column, parity and horizontal
            // neighbour offset for the whole pass; its row advances by
            // 64/(L/2) per pass, and all lanes move to the next replica group
            // together.  Only the up/down wraps are tested per pass.
            constexpr bool STEP_ROWS = LT > 0 && 64 % (LT / 2) == 0 && (64 / (LT / 2)) % 2 == 0 &&
                                       (LT * LT / 2) % 64 == 0;
            if (STEP_ROWS && (ub & 63) == 0 && ub < ue) {
                constexpr int RS = STEP_ROWS ? 64 / (LT / 2) : 0;   // rows per pass
                int gs = __builtin_amdgcn_readfirstlane(ub / nh);
                int kb = ub - gs * nh;   // lane 0's unit in its group: uniform, so the group change is too
                int k = kb + lane;
                int y = k / half;
                const int m = k - y * half;
                const int p = (y + colour) & 1;   // constant: y advances by an even count
                int mh = p ? m + 1 : m - 1;
                mh = mh < 0 ? half - 1 : (mh == half ? 0 : mh);
                const int dh = mh - m;
                int addr = gs * N + colour * nh + k;
                uint32_t n = (uint32_t)(y * L + 2 * m + p);
                for (int u0 = ub; u0 < ue; u0 += 64) {
                    const int ku = y == 0 ? k + nh - half : k - half;
                    const int kd = y + 1 == L ? k - nh + half : k + half;
                    chunk(u0 + lane < ue, gs, k, k + dh, ku, kd, addr, n);
                    kb += 64;
                    k += 64;
                    y += RS;
                    n += (uint32_t)(RS * L);
                    addr += 64;
                    if (kb >= nh) {   // every lane at once: the next replica group
                        kb -= nh;
                        k -= nh;
                        y -= L;
                        n -= (uint32_t)N;
                        addr += N - nh;
                        ++gs;
                    }
                }
            } else {
                for (int u0 = ub; u0 < ue; u0 += 64) {
                    const int u = u0 + lane;
                    const bool in = u < ue;
                    const int uu = in ? u : ub;   // any in-range unit; the chunk ignores it
                    const int gs = uu / nh, k = uu - gs * nh;
                    const int y = k / half, m = k - y * half;
                    const int p = (y + colour) & 1;
                    int mh = p ? m + 1 : m - 1;                  // the other horizontal neighbour
                    mh = mh < 0 ? half - 1 : (mh == half ? 0 : mh);
                    const int kh = k - m + mh;
                    const int ku = y == 0 ? k + nh - half : k - half;
                    const int kd = y + 1 == L ? k - nh + half : k + half;
                    chunk(in, gs, k, kh, ku, kd, gs * N + colour * nh + k, (uint32_t)(y * L + 2 * m + p));
                }
            }
            if (pool)
                sweep_sparse_pooled(lat, eu, en, ctl, h, dense, N, group0, Th, (uint32_t)i, c3, key0, key1,
                                    wcalls);
            else if (stream && G == 1) {
                stream_rounds<true>(q, 64, lat, eu + rb, en + rb, rcap, N, group0, tmask, (uint32_t)i, c3,
                                    key0, key1, wcalls);
                stream_tail<true>(q, lat, eu + rb, en + rb, rcap, N, group0, tmask, (uint32_t)i, c3, key0,
                                  key1, wcalls);
            } else if (stream) {
                stream_rounds<false>(q, 64, lat, eu + rb, en + rb, rcap, N, group0, tmask, (uint32_t)i, c3,
                                     key0, key1, wcalls);
                stream_tail<false>(q, lat, eu + rb, en + rb, rcap, N, group0, tmask, (uint32_t)i, c3, key0,
                                   key1, wcalls);
            }
            else
                sweep_sparse_wave(lat, eu + ub, en + ub, cnt, dense, N, group0, Th, (uint32_t)i, c3, key0,
                                  key1, wcalls);
        }
    }
    __syncthreads();
    for (int u = tid; u < G * N; u += T) {
        const int gs = u / N, n = u - gs * N;
        const int y = n / L, x = n - y * L;
        base[u] = lat[(size_t)gs * N + ((x + y) & 1) * nh + y * half + (x >> 1)];
    }
    // word-site updates and attempted flips of this wavefront's range, in
    // closed form: the item's sweeps x 2 colours x its units, 64 replicas
    // each except the valid ones of the last group
    const int mine = max(ue - ub, 0);
    const int nlast = max(ue - max(ub, (G - 1) * nh), 0);   // its units in the last group
    const uint64_t nsw = (uint64_t)(s_end - s_begin);
    const uint64_t nwords = nsw * 2u * (uint64_t)mine;
    const uint64_t nflips =
        nsw * 2u * ((uint64_t)(mine - nlast) * 64u + (uint64_t)nlast * (uint64_t)__popcll(vlast));
    flush_stats(stats, lane == 0 ? nwords : 0ull, lane == 0 ? wcalls : 0u, lane == 0 ? nflips : 0ull);
}

template <bool EA>
__device__ __forceinline__ void sweep_dispatch(const SweepItem &it, const RunInfo &R, const PopState &S,
                                               uint64_t *lds, int dense, unsigned long long *stats)
{
    switch (R.L) {
    case 8: sweep_item<8, EA, false>(it, R, S, lds, dense, stats); break;
    case 16: sweep_item<16, EA, false>(it, R, S, lds, dense, stats); break;
    case 24: sweep_item<24, EA, false>(it, R, S, lds, dense, stats); break;
    case 32: sweep_item<32, EA, false>(it, R, S, lds, dense, stats); break;
    case 48: sweep_item<48, EA, false>(it, R, S, lds, dense, stats); break;
    case 64: sweep_item<64, EA, false>(it, R, S, lds, dense, stats); break;
    case 128: sweep_item<128, EA, false>(it, R, S, lds, dense, stats); break;
    default: sweep_item<0, EA, false>(it, R, S, lds, dense, stats); break;
    }
}

// LS < 0: any lattice size and model, chosen per item; otherwise every item
// of the launch has L = LS and the model EA (a kernel of its own allocates
// only the registers that one size needs).
template <int LS, bool EA>
__device__ __forceinline__ void sweep_one(const SweepItem &it, const RunInfo *runs, const PopState *st,
                                          uint64_t *lds, uint32_t lds_bytes, int dense, unsigned long long *stats)
{
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S) || R.theta == 0) return;
    // an item that does not fit the LDS of this launch (a list that does not
    // belong to the launch's plan) is skipped and counted, never run
    if (msc_lds_need(R.N, it.ngroups, R.model == PA_EA_PMJ, (int)(blockDim.x >> 6),
                     LS >= 0 ? dense : dense | MSC_WHOLE_LISTS) > lds_bytes) {
        if (threadIdx.x == 0) atomicAdd(&stats[ST_STALL], 1ull);
        return;
    }
    if constexpr (LS >= 0) {
        sweep_item<LS, EA, true>(it, R, S, lds, dense, stats);
    } else {
        if (R.model == PA_EA_PMJ) sweep_dispatch<true>(it, R, S, lds, dense, stats);
        else sweep_dispatch<false>(it, R, S, lds, dense, stats);
    }
}

// One workgroup per item, or (queue != nullptr) a persistent grid whose
// workgroups take items in list order from a ticket counter.  The items are
// listed largest first, so the last tickets are the cheapest.  queue[0] is
// the next ticket, queue[1] counts workgroups that found the list empty; the
// last of them resets both, so the next launch (or graph replay) starts
// from zero without a separate clear.
//
// Sweep chunks (persistent grid only): an item may cover a part of its
// groups' theta sweeps.  The list holds every first chunk before any second
// one, and so on, so the chunk an item depends on was taken from the queue
// earlier, by a workgroup that is running or done.  When a chunk has stored
// its lattices, its workgroup publishes (launch generation << 4 | chunk + 1)
// in the groups' flag slot; the next chunk waits for that value before it
// loads them.  queue[2] is the launch generation: every workgroup reads it
// before taking a ticket, and the last one to leave increments it, so
// values left by earlier launches or graph replays never match.  The wait
// ends because the producer holds an earlier ticket; it is bounded all the
// same, and a wait that runs out is counted in the stall counter (the
// results of that step are then not trustworthy, and reading the work
// counters reports it).
constexpr unsigned int SWEEP_WAIT_SPINS = 1u << 22;

template <int LS, bool EA>
__global__ void __launch_bounds__(1024) k_sweep_msc(const SweepItem *items, int n_items, const RunInfo *runs,
                                                    const PopState *st, int dense, unsigned long long *stats,
                                                    unsigned int *queue, unsigned int *flags, uint32_t lds_bytes)
{
    extern __shared__ uint64_t lds[];
    if (queue == nullptr) {
        sweep_one<LS, EA>(items[blockIdx.x], runs, st, lds, lds_bytes, dense, stats);
        return;
    }
    __shared__ unsigned int ticket, gen;
    if (threadIdx.x == 0) gen = __hip_atomic_load(&queue[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) ticket = atomicAdd(&queue[0], 1u);
        __syncthreads();
        const unsigned int t = ticket;
        if (t >= (unsigned int)n_items) break;
        const SweepItem it = items[t];
        if (it.chunk > 0) {
            if (threadIdx.x == 0) {
                const unsigned int want = (gen << 4) | (unsigned int)it.chunk;
                unsigned int spins = 0;
                while (__hip_atomic_load(&flags[it.base], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
                    if (++spins == SWEEP_WAIT_SPINS) {
                        atomicAdd(&stats[ST_STALL], 1ull);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
        }
        sweep_one<LS, EA>(it, runs, st, lds, lds_bytes, dense, stats);
        if (it.chunk + 1 < it.nchunk) {
            // every wavefront waits for its own lattice stores (a barrier
            // alone does not), so that the release by the first thread,
            // which writes this XCD's L2 back, covers all of them
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&flags[it.base], (gen << 4) | (unsigned int)(it.chunk + 1), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1u) == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
            atomicAdd(&queue[2], 1u);
        }
    }
}

// -------------------------------------------------------------- step (v)

// Partner words of the permutation pairing ([group][site] u64): the spare
// spin buffer of population 0 (its previous population is no longer needed
// once the step's copies are done; it holds at least 8 bytes per site and
// group in either layout).
__device__ __forceinline__ uint8_t *wang_partner_words(const RunInfo &R, const PopState &S)
{
    return R.spins[0][S.cur ^ 1];
}

// Word of 64 replicas of group g at site n, from either layout.
template <int REPR>
__device__ __forceinline__ uint64_t load_word(const uint8_t *buf, int g, int n, int N)
{
    if (REPR == PA_MSC64) return ((const uint64_t *)buf)[(size_t)g * N + n];
    const uint4 *q = (const uint4 *)(buf + ((size_t)g * N + n) * 64);
    uint4 v[4] = {q[0], q[1], q[2], q[3]};
    return pack64(v);
}

// Measurement of replica groups (64 replicas each).  A workgroup of
// MEAS_WAVES wavefronts takes a measure item of consecutive groups of one
// (run, pop); each group gets meas_waves_per_group(N) wavefronts, which
// split its sites 64 at a time.  A lane accumulates, in bit-sliced
// counters over its sites, the per-replica numbers of unsatisfied bonds
// (E = 2 #unsat - 2N), down spins (M = N - 2 #down), and for overlap pairs
// the Hamming distance (Q = N - 2 d) and the number of bonds whose product
// differs (Q_l = 2N - 2 d_l); neighbour words are read straight from
// memory (the lattice block of a group is contiguous, so they hit the
// caches).  The counters are turned into per-replica integers by
// transposes, the wavefronts of a group are summed in LDS, the energies are
// stored, and the group's integer sums go to its slot of the partial-sum
// array; k_meas_chunk reduces those per chunk.
template <int REPR, int LT, bool WITH_Q>
__device__ __forceinline__ void measure_group(const SweepItem &it, int g, int sub, int wpg, bool live,
                                              const RunInfo &R, const PopState &S, const PopState *st,
                                              uint32_t (*red)[MEAS_WAVES][64], const uint64_t *lw)
{
    // the group's own words come from LDS when the workgroup staged them
    // (lw != nullptr), else from memory
    auto own = [&](int gg, int n, int NN) -> uint64_t {
        return lw ? lw[n] : load_word<REPR>(R.spins[it.pop][S.cur], gg, n, NN);
    };
    const int L = LT ? LT : R.L;
    const int N = L * L;
    const int Rc = S.Rcur;
    const int lane = threadIdx.x & 63, wv = wave_id();
    const uint8_t *buf = R.spins[it.pop][S.cur];
    // overlap partners of this group's replicas
    int mode = 0;                      // 0 none, 1 index shift, 2 two populations, 3 permutation pairs
    uint64_t pairmask = 0;
    const uint8_t *pbuf = buf;
    int pg = 0, sh = 0;
    const int pgroups = R.groups_cap;
    if (!WITH_Q) {
        // no run of the launch measures overlaps
    } else if (live && R.overlap == PA_Q_INDEX_SHIFT) {
        const int h = Rc >> 1;
        const int lo = g * 64;
        if (lo < h) {
            mode = 1;
            const int cntp = min(64, h - lo);
            pairmask = cntp >= 64 ? ~0ull : ((1ull << cntp) - 1);
            pg = (lo + h) >> 6;
            sh = (lo + h) & 63;
        }
    } else if (live && R.overlap == PA_Q_TWO_POP && it.pop == 0) {
        const PopState &S1 = st[it.run * MAX_POP + 1];
        if (pop_active(S1)) {
            const int m = min(Rc, S1.Rcur);
            const int lo = g * 64;
            if (lo < m) {
                mode = 2;
                const int cntp = min(64, m - lo);
                pairmask = cntp >= 64 ? ~0ull : ((1ull << cntp) - 1);
                pbuf = R.spins[1][S1.cur];
                pg = g;
            }
        }
    } else if (live && is_wang(R.overlap) && wang_bufs(R.wang, R.R_cap, R.wang_lb).hdr[0] == 0) {
        // permutation pairs (j, pi_j) for every replica: the partners'
        // configurations were gathered into bit-packed words (k_wang_gather)
        mode = 3;
        const int cntp = min(64, Rc - g * 64);
        pairmask = cntp >= 64 ? ~0ull : ((1ull << cntp) - 1);
        pbuf = wang_partner_words(R, S);
        pg = g;
    }
    if (R.exact_dos && S.i > 0) {
        // theta = infinity: the energies were drawn (k_dos_sample); only
        // their sums and minimum are recorded.  One barrier, as below.
        __syncthreads();
        if (!live || sub != 0) return;
        const int j = g * 64 + lane;
        const bool valid = j < Rc;
        const int64_t E = valid ? R.E[it.pop][S.cur][j] : 0;
        int64_t part[MEAS_PART];
        part[0] = wave_sum<int64_t>(E);
        part[1] = wave_sum<int64_t>(E * E);
        for (int k = 2; k < MEAS_PART - 1; ++k) part[k] = 0;
        part[MEAS_PART - 1] = wave_min(valid ? (int)E : INT32_MAX);
        if (lane < MEAS_PART) {
            int64_t mine = 0;
#pragma unroll
            for (int k = 0; k < MEAS_PART; ++k)
                if (lane == k) mine = part[k];
            R.part[it.pop][(size_t)g * MEAS_PART + lane] = mine;
        }
        return;
    }
    uint32_t totU = 0, totD = 0, totH = 0, totK = 0;
    // every lane of the wavefront runs the same iterations (flushes are
    // wave-wide).  Counts are flushed after every block of 16 sites per lane
    // (at most 2 per site: 32 < 2^VB); mode is uniform over the wavefront, so
    // are the overlap counts.
    if constexpr (WITH_Q) {
        // four counters: the incremental form keeps the loop within the
        // registers of four wavefronts per SIMD
        uint64_t cU[VB] = {}, cD[VB] = {}, cH[VB] = {}, cK[VB] = {};
        for (int b0 = 64 * sub; b0 < N; b0 += 16 * 64 * wpg) {
            // sites per lane in this block of 16 (uniform): bounds the counts
            const int tsites = min(16, (N - b0 + 64 * wpg - 1) / (64 * wpg));
#pragma unroll 4
            for (int t = 0; t < 16; ++t) {
                const int n = b0 + t * 64 * wpg + lane;
                if (live && n < N) {
                    const int y = n / L, x = n - y * L;
                    const int nr = y * L + (x + 1 == L ? 0 : x + 1);
                    const int nd = (y + 1 == L ? 0 : y + 1) * L + x;
                    const uint8_t jn = R.jbits[n];
                    const uint64_t w = own(g, n, N);
                    const uint64_t wr = own(g, nr, N);
                    const uint64_t wd = own(g, nd, N);
                    const uint64_t br = w ^ wr, bd = w ^ wd;
                    vinc2(cU, br ^ ((jn & 1) ? ~0ull : 0ull), bd ^ ((jn & 2) ? ~0ull : 0ull));
                    vinc(cD, w);
                    if (mode) {
                        uint64_t q, qr, qd;
                        if (mode == 3) {
                            const uint64_t *pw = (const uint64_t *)pbuf + (size_t)pg * N;
                            q = pw[n];
                            qr = pw[nr];
                            qd = pw[nd];
                        } else if (mode == 1 && sh) {
                            const bool two = pg + 1 < pgroups;
                            q = (load_word<REPR>(buf, pg, n, N) >> sh) |
                                (two ? load_word<REPR>(buf, pg + 1, n, N) << (64 - sh) : 0ull);
                            qr = (load_word<REPR>(buf, pg, nr, N) >> sh) |
                                 (two ? load_word<REPR>(buf, pg + 1, nr, N) << (64 - sh) : 0ull);
                            qd = (load_word<REPR>(buf, pg, nd, N) >> sh) |
                                 (two ? load_word<REPR>(buf, pg + 1, nd, N) << (64 - sh) : 0ull);
                        } else {
                            q = load_word<REPR>(pbuf, pg, n, N);
                            qr = load_word<REPR>(pbuf, pg, nr, N);
                            qd = load_word<REPR>(pbuf, pg, nd, N);
                        }
                        vinc(cH, w ^ q);
                        vinc2(cK, br ^ q ^ qr, bd ^ q ^ qd);
                    }
                }
            }
            const int p1 = planes_for(tsites), p2 = planes_for(2 * tsites);
            totU += vflush(cU, p2);
            totD += vflush(cD, p1);
            if (mode) {
                totH += vflush(cH, p1);
                totK += vflush(cK, p2);
            }
        }
    } else {
        // energies and magnetisations only: carry-save counting
        const bool ea = R.model == PA_EA_PMJ;      // the ferromagnet's bond signs are all +1
        const int gl = live ? g : it.group0;       // a group that exists, for lanes that drop their loads
        for (int b0 = 64 * sub; b0 < N; b0 += 16 * 64 * wpg) {
            const int tsites = min(16, (N - b0 + 64 * wpg - 1) / (64 * wpg));
            Csa2 cU;
            Csa1 cD;
            // U sites at a time, all their loads issued before the first use
            // and none behind a branch (a wavefront or lane with no site
            // there loads one that exists and drops it); the carries of
            // weight 4 and up pair up on uniform branches
            constexpr int U = REPR == PA_MSC64 ? 4 : 2;
#pragma unroll 1
            for (int t0 = 0; t0 < 16; t0 += U) {
                uint64_t w[U], wr[U], wd[U];
                uint32_t jn[U];
                bool ok[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int n = b0 + (t0 + u) * 64 * wpg + lane;
                    ok[u] = live && n < N;
                    const int nn = ok[u] ? n : 0;
                    const int y = nn / L, x = nn - y * L;
                    const int nr = y * L + (x + 1 == L ? 0 : x + 1);
                    const int nd = (y + 1 == L ? 0 : y + 1) * L + x;
                    jn[u] = ea ? R.jbits[nn] : 0u;
                    w[u] = own(gl, nn, N);
                    wr[u] = own(gl, nr, N);
                    wd[u] = own(gl, nd, N);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t z = ok[u] ? ~0ull : 0ull;   // zero inputs past the last site
                    const uint64_t ur = (w[u] ^ wr[u] ^ ((jn[u] & 1) ? ~0ull : 0ull)) & z;
                    const uint64_t ud = (w[u] ^ wd[u] ^ ((jn[u] & 2) ? ~0ull : 0ull)) & z;
                    cU.add(t0 + u, ur, ud);
                    cD.add(t0 + u, w[u] & z);
                }
            }
            uint64_t pl[VB];
            cU.planes(pl);
            totU += vflush(pl, planes_for(2 * tsites));
            cD.planes(pl);
            totD += vflush(pl, planes_for(tsites));
        }
    }
    if (wpg > 1) {
        red[0][wv][lane] = totU;
        red[1][wv][lane] = totD;
        red[2][wv][lane] = totH;
        red[3][wv][lane] = totK;
    }
    __syncthreads();
    if (!live || sub != 0) return;
    uint32_t U = totU, D = totD, H = totH, Kc = totK;
    for (int k = 1; k < wpg; ++k) {
        U += red[0][wv + k][lane];
        D += red[1][wv + k][lane];
        H += red[2][wv + k][lane];
        Kc += red[3][wv + k][lane];
    }
    const int j = g * 64 + lane;
    const bool valid = j < Rc;
    const int64_t E = 2 * (int64_t)U - 2 * (int64_t)N;
    const int64_t M = R.exact_dos ? 0 : (int64_t)N - 2 * (int64_t)D;   // energies only at theta = infinity
    if (valid) R.E[it.pop][S.cur][j] = (int32_t)E;
    const int64_t v = valid ? 1 : 0;
    const bool pair = mode && ((pairmask >> lane) & 1u);
    const int64_t pv = pair ? 1 : 0;
    const int64_t Q = (int64_t)N - 2 * (int64_t)H, Ql = 2 * (int64_t)N - 2 * (int64_t)Kc;
    int64_t part[MEAS_PART];
    part[0] = wave_sum<int64_t>(v * E);
    part[1] = wave_sum<int64_t>(v * E * E);
    part[2] = wave_sum<int64_t>(v * (M < 0 ? -M : M));
    part[3] = wave_sum<int64_t>(v * M * M);
    part[4] = wave_sum<int64_t>(pv);
    part[5] = wave_sum<int64_t>(pv * Q);
    part[6] = wave_sum<int64_t>(pv * (Q < 0 ? -Q : Q));
    part[7] = wave_sum<int64_t>(pv * Q * Q);
    part[8] = wave_sum<int64_t>(pv * Ql);
    part[9] = wave_sum<int64_t>(pv * Ql * Ql);
    part[10] = wave_min(valid ? (int)E : INT32_MAX);
    if (pair && R.qhist) {
        const size_t Np1 = (size_t)N + 1;
        atomicAdd(&R.qh[((size_t)it.pop * R.K + S.i) * Np1 + H], 1);
        if (R.overlap == PA_Q_TWO_POP) atomicAdd(&R.qh[((size_t)1 * R.K + S.i) * Np1 + H], 1);
    }
    if (lane < MEAS_PART) {
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < MEAS_PART; ++k)
            if (lane == k) mine = part[k];
        R.part[it.pop][(size_t)g * MEAS_PART + lane] = mine;
    }
}

template <int REPR, bool WITH_Q>
__global__ void __launch_bounds__(MEAS_THREADS) k_measure(const SweepItem *items, const RunInfo *runs,
                                                          const PopState *st)
{
    __shared__ uint32_t red[4][MEAS_WAVES][64];
    extern __shared__ uint64_t words[];   // [groups of the item][N] when staged
    const SweepItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int wpg = meas_waves_per_group(R.N);
    const int wv = wave_id();
    const int k = wv / wpg, sub = wv - k * wpg;
    const int g = it.group0 + k;
    const bool live = k < it.ngroups && g * 64 < S.Rcur;
    // int8 layout: each group's words are read once from memory into LDS
    // (four 16-byte loads per site, packed on the way), then every site reads
    // itself and its neighbours from there instead of loading and packing
    // three 64-byte rows.  Not for lattices above MEAS_STAGE_N sites, nor at
    // theta = infinity (no lattice to read).  The bit-packed layout reads its
    // 8-byte words straight from memory: staging them measured slower (34
    // against 22 us at L = 64, R = 1e5), the barrier after the staging pass
    // keeping loads and counting from overlapping.
    const bool staged = REPR == PA_INT8 && R.N <= MEAS_STAGE_N && !(R.exact_dos && S.i > 0);
    const uint64_t *lw = nullptr;
    if (staged) {
        uint64_t *mine = words + (size_t)k * R.N;
        if (live) {
            const uint8_t *buf = R.spins[it.pop][S.cur];
            for (int n = sub * 64 + (threadIdx.x & 63); n < R.N; n += 64 * wpg)
                mine[n] = load_word<REPR>(buf, g, n, R.N);
        }
        __syncthreads();
        lw = mine;
    }
    switch (R.L) {
    case 8: measure_group<REPR, 8, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    case 16: measure_group<REPR, 16, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    case 24: measure_group<REPR, 24, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    case 32: measure_group<REPR, 32, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    case 48: measure_group<REPR, 48, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    case 64: measure_group<REPR, 64, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    default: measure_group<REPR, 0, WITH_Q>(it, g, sub, wpg, live, R, S, st, red, lw); break;
    }
}

// ----------------------------------------------- theta = infinity draws
//
// Step (iv) in the theta = infinity limit (Sec. V C): every replica's energy
// is an independent draw from the exact distribution at beta_i.  One thread
// per replica (a wavefront per replica group): a 64-bit Philox draw and a
// binary search over the level thresholds C[i][0..N] (non-decreasing) for
// the first level with v < C_m, the top level if there is none.
__global__ void __launch_bounds__(256) k_dos_sample(const Item *items, int n_items, const RunInfo *runs,
                                                    const PopState *st)
{
    const int idx = blockIdx.x * 4 + wave_id(), lane = threadIdx.x & 63;
    if (idx >= n_items) return;
    const Item it = items[idx];
    const RunInfo &R = runs[it.run];
    if (!R.exact_dos) return;
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int j = it.group * 64 + lane;
    if (j >= S.Rcur) return;
    const int N = R.N, i = S.i;
    const u32x4 o = philox10((uint32_t)j, 0u, (uint32_t)i, (TAG_DOS << 28) | ((uint32_t)it.pop << 24), R.key0,
                             R.key1);
    const uint64_t v = (uint64_t)o.x | ((uint64_t)o.y << 32);
    const uint64_t *C = R.tabD + (size_t)i * (N + 1);
    int lo = 0, hi = N + 1;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (v < C[m]) hi = m;
        else lo = m + 1;
    }
    R.E[it.pop][S.cur][j] = -2 * N + 4 * min(lo, N);
}

// ---------------------------------------------- permutation pairing (q)
//
// Sec. III D, pairings from permutations (Wang et al.), for runs with
// PA_Q_WANG / PA_Q_WANG_RDM, before the measurement of every temperature:
//   k_wang_pairs   one workgroup per run: the permutations and the repair;
//   k_wang_rows    the population as bit rows, one per replica;
//   k_wang_gather  the partners' configurations as bit-packed words;
// then k_measure takes the pairs (j, pi_j) like any other overlap pairs.
//
// The random permutations are index orders of 64-bit Philox keys: a key's
// top bits pick one of B >= R_i buckets (a power of two, so about one key
// per bucket), the bucket counts are scanned into starts, the indices are
// scattered into their buckets, and an index's rank is its bucket's start
// plus the members of the bucket with a smaller (key, index).  The repair is
// serial by nature: the mismatched positions are listed in search order,
// then one wavefront takes them in turn and finds each exchange partner
// with a 64-wide search (a ballot over consecutive candidates).  With the
// identity search pattern the candidates inside the mismatched replica's
// own family, which is one run of equal labels, are skipped without being
// tested: none of them can qualify.  Data that other wavefronts wrote in
// the same launch is read with device-coherent loads after the writers have
// waited for their stores.

constexpr int WANG_THREADS = 1024;

__device__ __forceinline__ int32_t ldc(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void stc(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier after which every wavefront's earlier stores have completed.
__device__ __forceinline__ void wg_sync_stores()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Key of index k for the pairing at temperature i: words 0-1 (pi) or 2-3
// (the search pattern) of Philox(seed; k, 0, i, TAG_PERM << 28).
__device__ __forceinline__ uint64_t perm_key(int k, int i, int which, uint32_t key0, uint32_t key1)
{
    const u32x4 o = philox10((uint32_t)k, 0u, (uint32_t)i, TAG_PERM << 28, key0, key1);
    return which == 0 ? ((uint64_t)o.x | ((uint64_t)o.y << 32)) : ((uint64_t)o.z | ((uint64_t)o.w << 32));
}

// Exclusive prefix over the workgroup of one value per thread; *total gets
// the sum.  sh: 17 ints of LDS.
__device__ int block_scan_excl(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, wv = wave_id(), nw = blockDim.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = sh[w];
            sh[w] = a;
            a += t;
        }
        sh[16] = a;
    }
    __syncthreads();
    const int r = sh[wv] + x - v;
    *total = sh[16];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(WANG_THREADS) k_wang_pairs(const RunInfo *runs, const PopState *st, int run0,
                                                              int lds_ints)
{
    __shared__ int sh[17];
    __shared__ int big;
    extern __shared__ int32_t wlds[];   // lds_ints: labels and partner labels when they fit
    const int run = run0 + blockIdx.x;
    const RunInfo &R = runs[run];
    if (!is_wang(R.overlap)) return;
    const PopState &S = st[run * MAX_POP];
    if (!pop_active(S)) return;
    const int Rc = S.Rcur, i = S.i;
    const int T = blockDim.x, tid = threadIdx.x;
    const int32_t *fam = R.fam[0][S.cur];
    const WangBufs W = wang_bufs(R.wang, R.R_cap, R.wang_lb);
    const bool rdm = R.overlap == PA_Q_WANG_RDM;
    const uint32_t key0 = R.key0, key1 = R.key1;
    // A family of more than Rc / 2 replicas (then no valid pairing exists)
    // covers the middle index: it is one run of equal labels.
    if (tid == 0) {
        const int h = Rc >> 1, f = fam[h];
        int lo = 0, hi = h;
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (fam[m] < f) lo = m + 1;
            else hi = m;
        }
        const int first = lo;
        lo = h + 1;
        hi = Rc;
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (fam[m] <= f) lo = m + 1;
            else hi = m;
        }
        big = 2 * (int64_t)(lo - first) > (int64_t)Rc ? 1 : 0;
        if (big) stc(&W.hdr[0], 1);
    }
    __syncthreads();
    if (big) return;

    int lbc = 1;
    while ((1 << lbc) < Rc) ++lbc;
    const int B = 1 << lbc, shift = 64 - lbc;
    for (int which = 0; which < (rdm ? 2 : 1); ++which) {
        int32_t *out = which == 0 ? W.pi : W.sigma;
        for (int b = tid; b < B; b += T) stc(&W.cnt[b], 0);
        wg_sync_stores();
        for (int k = tid; k < Rc; k += T) atomicAdd(&W.cnt[perm_key(k, i, which, key0, key1) >> shift], 1);
        wg_sync_stores();
        const int seg = (B + T - 1) / T;
        const int b0 = min(B, tid * seg), b1 = min(B, b0 + seg);
        int sum = 0;
        for (int b = b0; b < b1; ++b) sum += ldc(&W.cnt[b]);
        int total;
        int acc = block_scan_excl(sum, sh, &total);
        for (int b = b0; b < b1; ++b) {
            const int c = ldc(&W.cnt[b]);
            stc(&W.start[b], acc);
            stc(&W.cnt[b], acc);   // fill cursor of the bucket
            acc += c;
        }
        if (tid == 0) stc(&W.start[B], Rc);
        wg_sync_stores();
        for (int k = tid; k < Rc; k += T) {
            const int b = (int)(perm_key(k, i, which, key0, key1) >> shift);
            stc(&W.members[atomicAdd(&W.cnt[b], 1)], k);
        }
        wg_sync_stores();
        for (int k = tid; k < Rc; k += T) {
            const uint64_t kk = perm_key(k, i, which, key0, key1);
            const int b = (int)(kk >> shift);
            const int lo = ldc(&W.start[b]), hi = ldc(&W.start[b + 1]);
            int r = lo;
            for (int q = lo; q < hi; ++q) {
                const int m = ldc(&W.members[q]);
                if (m == k) continue;
                const uint64_t km = perm_key(m, i, which, key0, key1);
                r += (km < kk || (km == kk && m < k)) ? 1 : 0;
            }
            stc(&out[r], k);
        }
        wg_sync_stores();
    }

    // families of the initial partners, and the mismatched positions in
    // search order (ascending)
    for (int k = tid; k < Rc; k += T) stc(&W.fampi[k], fam[ldc(&W.pi[k])]);
    wg_sync_stores();
    const int seg = (Rc + T - 1) / T;
    const int t0 = min(Rc, tid * seg), t1 = min(Rc, t0 + seg);
    int mine = 0;
    for (int t = t0; t < t1; ++t) {
        const int k = rdm ? ldc(&W.sigma[t]) : t;
        mine += ldc(&W.fampi[k]) == fam[k] ? 1 : 0;
    }
    int nlist;
    int pos = block_scan_excl(mine, sh, &nlist);
    for (int t = t0; t < t1; ++t) {
        const int k = rdm ? ldc(&W.sigma[t]) : t;
        if (ldc(&W.fampi[k]) == fam[k]) stc(&W.list[pos++], t);
    }
    wg_sync_stores();
    // When 2 R_i ints fit the workgroup's LDS, the repair reads and writes
    // the family labels and the partners' labels there, and logs its
    // exchanges (in the bucket arrays, free by now) instead of applying them
    // to pi in global memory; they are replayed onto pi in LDS at the end.
    const bool in_lds = 2 * Rc <= lds_ints;
    int32_t *Lfam = wlds, *Lfpi = wlds + Rc;
    if (in_lds) {
        for (int k = tid; k < Rc; k += T) {
            Lfam[k] = fam[k];
            Lfpi[k] = ldc(&W.fampi[k]);
        }
        __syncthreads();
    }
    // The other wavefronts wait for the repair, then load and store pi with
    // it (the replay of the exchanges itself is one wavefront's, in order).
    int nsw = 0, status = 0;
    int32_t *swaps = W.cnt;   // [2 B + 1] ints, B >= R_i: room for R_i exchanges
    // IN_LDS (a constant in each copy of the repair): the labels are read
    // with LDS instructions only, not through generic pointers that would
    // make every probe wait for both memory counters.  Values of one lane
    // that the whole wavefront needs are read with readlane (the lane index
    // is uniform), not with a permute through LDS.
    auto repair = [&](auto in_lds_c) {
        constexpr bool IN_LDS = decltype(in_lds_c)::value;
        auto famv = [&](int m) {
            if constexpr (IN_LDS) return Lfam[m];
            else return fam[m];
        };
        auto fpiv = [&](int m) {
            if constexpr (IN_LDS) return Lfpi[m];
            else return ldc(&W.fampi[m]);
        };

        // The repair, one wavefront, over the list in batches of 64 entries.
        // What does not change during the repair (position, its place in the
        // search order, its family, the end of its family's run of labels, its
        // initial partner) is loaded for a whole batch at once; an entry is
        // still open unless an earlier exchange in this repair took its
        // position as the partner (an exchange leaves both of its positions
        // matched for good), which the lanes track by comparing positions.
        // With the identity pattern the mismatches of one family come one after
        // the other, and a candidate that failed for one of them fails for the
        // next as well (exchanges only hand this family's replicas to
        // candidates), so the search resumes after the previous partner
        // (unwrapped candidate index prev_u).
        const int lane = tid;
        int prev_f = -1;
        int64_t prev_u = 0;
        for (int e0 = 0; e0 < nlist && status == 0; e0 += 64) {
            const int e = e0 + lane;
            int t_l = 0, k_l = -1, f_l = 0, hi_l = 0, p_l = 0;
            bool open_l = false;
            if (e < nlist) {
                t_l = ldc(&W.list[e]);
                k_l = rdm ? ldc(&W.sigma[t_l]) : t_l;
                f_l = famv(k_l);
                open_l = fpiv(k_l) == f_l;
                if (!IN_LDS) p_l = ldc(&W.pi[k_l]);
                if (!rdm) {   // the first later index with another label
                    int lo = t_l + 1, hi = Rc;
                    while (lo < hi) {
                        const int m = (lo + hi) >> 1;
                        if (famv(m) == f_l) lo = m + 1;
                        else hi = m;
                    }
                    hi_l = lo;
                }
            }
            const int nb = min(64, nlist - e0);
            for (int j = 0; j < nb; ++j) {
                if (!__builtin_amdgcn_readlane((int)open_l, j)) continue;
                const int t = __builtin_amdgcn_readlane(t_l, j), k = __builtin_amdgcn_readlane(k_l, j);
                const int fk = __builtin_amdgcn_readlane(f_l, j), pk = __builtin_amdgcn_readlane(p_l, j);
                int64_t u = t + 1;
                if (!rdm) {
                    u = __builtin_amdgcn_readlane(hi_l, j);
                    if (fk == prev_f && prev_u + 1 > u) u = prev_u + 1;
                }
                const int64_t uend = (int64_t)t + Rc;   // candidates t + 1 .. t + Rc - 1, indices mod Rc
                int found = -1, fm = 0;
                for (; u < uend; u += 64) {
                    const int64_t uu = u + lane;
                    bool ok = false;
                    int m = 0, fpm = 0;
                    if (uu < uend) {
                        const int q = (int)(uu >= Rc ? uu - Rc : uu);
                        m = rdm ? ldc(&W.sigma[q]) : q;
                        fpm = fpiv(m);
                        ok = famv(m) != fk && fpm != fk;
                    }
                    const uint64_t bal = __ballot(ok);
                    if (bal) {
                        const int first = __ffsll((unsigned long long)bal) - 1;
                        found = __builtin_amdgcn_readlane(m, first);
                        fm = __builtin_amdgcn_readlane(fpm, first);
                        prev_u = u + first;
                        break;
                    }
                }
                if (found < 0) {   // impossible with no family above Rc / 2
                    status = 2;
                    break;
                }
                if constexpr (IN_LDS) {
                    if (lane == 0) {
                        Lfpi[k] = fm;
                        Lfpi[found] = fk;
                        swaps[2 * nsw] = k;
                        swaps[2 * nsw + 1] = found;
                    }
                    ++nsw;
                } else {
                    if (lane == 0) {
                        const int pm = ldc(&W.pi[found]);
                        stc(&W.pi[k], pm);
                        stc(&W.pi[found], pk);
                        stc(&W.fampi[k], fm);
                        stc(&W.fampi[found], fk);
                    }
                    __builtin_amdgcn_s_waitcnt(0);
                }
                if (k_l == found) open_l = false;
                prev_f = fk;
            }
        }
        if (lane == 0) {
            sh[0] = nsw;
            sh[1] = status;
        }
    };
    if (tid < 64) {
        if (in_lds) repair(std::true_type{});
        else repair(std::false_type{});
    }
    __syncthreads();
    nsw = sh[0];
    status = sh[1];
    if (in_lds && status == 0) {   // replay the exchanges onto pi, in LDS
        int32_t *Lpi = Lfam;       // the family labels are no longer needed
        for (int k = tid; k < Rc; k += T) Lpi[k] = ldc(&W.pi[k]);
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            __builtin_amdgcn_s_waitcnt(0);   // this wavefront's exchange log is written
            for (int s0 = 0; s0 < nsw; s0 += 64) {
                int a = 0, b = 0;
                if (s0 + lane < nsw) {
                    a = ldc(&swaps[2 * (s0 + lane)]);
                    b = ldc(&swaps[2 * (s0 + lane) + 1]);
                }
                const int ns = min(64, nsw - s0);
                for (int j = 0; j < ns; ++j) {
                    const int x = __builtin_amdgcn_readlane(a, j), y = __builtin_amdgcn_readlane(b, j);
                    if (lane == 0) {
                        const int px = Lpi[x], py = Lpi[y];
                        Lpi[x] = py;
                        Lpi[y] = px;
                    }
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < Rc; k += T) stc(&W.pi[k], Lpi[k]);
    }
    if (tid == 0) {
        stc(&W.hdr[0], status);
        stc(&W.hdr[1], nlist);
    }
}

// Calibration: two independent chains of Philox calls per lane, all in
// registers (the outputs feed the next call's counter); an empty statement
// keeps the final values alive without a memory write.
__global__ void __launch_bounds__(256) k_philox_rate(int calls, uint32_t k0, uint32_t k1)
{
    uint32_t a0 = threadIdx.x, a1 = blockIdx.x, a2 = 0, a3 = 1;
    uint32_t b0 = threadIdx.x ^ 0x9E3779B9u, b1 = blockIdx.x, b2 = 2, b3 = 3;
    for (int k = 0; k < calls; ++k) {
        const u32x4 x = philox10(a0, a1, a2, a3, k0, k1);
        const u32x4 y = philox10(b0, b1, b2, b3, k0, k1);
        a0 = x.x; a1 = x.y; a2 = x.z; a3 = x.w;
        b0 = y.x; b1 = y.y; b2 = y.z; b3 = y.w;
    }
    asm volatile("" ::"v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(b0), "v"(b1), "v"(b2), "v"(b3));
}

hipError_t launch_philox_rate(int calls, hipStream_t s, int *blocks, int *threads)
{
    *blocks = 2048;
    *threads = 256;
    k_philox_rate<<<*blocks, *threads, 0, s>>>(calls, 0x01234567u, 0x89ABCDEFu);
    return hipGetLastError();
}

hipError_t prepare_wang_lds(size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_wang_pairs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

__device__ __forceinline__ bool wang_group_live(const Item &it, const RunInfo &R, const PopState &S)
{
    return is_wang(R.overlap) && it.pop == 0 && pop_active(S) && it.group * 64 < S.Rcur &&
           wang_bufs(R.wang, R.R_cap, R.wang_lb).hdr[0] == 0;
}

// Bit rows of population 0: word blk * 64 groups_cap + j holds, in bit s,
// the spin of replica j at site 64 blk + s.  One wavefront per replica
// group: lane s takes the word of site 64 blk + s (64 replicas), and a
// 64 x 64 transpose turns the 64 site words into the group's 64 rows.
template <int REPR>
__global__ void __launch_bounds__(256) k_wang_rows(const Item *items, int n_items, const RunInfo *runs,
                                                   const PopState *st)
{
    const int idx = blockIdx.x * 4 + wave_id(), lane = threadIdx.x & 63;
    if (idx >= n_items) return;
    const Item it = items[idx];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP];
    if (!wang_group_live(it, R, S)) return;
    const int N = R.N, g = it.group, nb = (N + 63) / 64;
    const size_t R64 = (size_t)R.groups_cap * 64;
    uint64_t *rows = wang_rows(R.wang, R.R_cap) + (size_t)g * 64 + lane;
    const uint8_t *buf = R.spins[0][S.cur];
#pragma unroll 4
    for (int blk = 0; blk < nb; ++blk) {
        const int n = blk * 64 + lane;
        const uint64_t w = n < N ? load_word<REPR>(buf, g, n, N) : 0ull;
        rows[(size_t)blk * R64] = transpose64(w);
    }
}

// Partner words: bit b of word (g, n) is the spin at site n of the partner
// pi_j of replica j = 64 g + b.  One wavefront per group: lane b reads its
// partner's bit row one 64-site block at a time, and a transpose turns the
// 64 rows into the block's 64 site words.  Lanes past R_i read replica 0
// (their bits are never used).
__global__ void __launch_bounds__(256) k_wang_gather(const Item *items, int n_items, const RunInfo *runs,
                                                     const PopState *st)
{
    const int idx = blockIdx.x * 4 + wave_id(), lane = threadIdx.x & 63;
    if (idx >= n_items) return;
    const Item it = items[idx];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP];
    if (!wang_group_live(it, R, S)) return;
    const int N = R.N, g = it.group, nb = (N + 63) / 64;
    const size_t R64 = (size_t)R.groups_cap * 64;
    const WangBufs W = wang_bufs(R.wang, R.R_cap, R.wang_lb);
    const int j = g * 64 + lane;
    const int p = j < S.Rcur ? W.pi[j] : 0;
    const uint64_t *rows = wang_rows(R.wang, R.R_cap) + p;
    uint64_t *dst = (uint64_t *)wang_partner_words(R, S) + (size_t)g * N;
#pragma unroll 4
    for (int blk = 0; blk < nb; ++blk) {
        const uint64_t col = transpose64(rows[(size_t)blk * R64]);
        const int n = blk * 64 + lane;
        if (n < N) dst[n] = col;
    }
}

// Per chunk of CH replicas (CH / 64 groups): the groups' partial sums, and
// the family statistics.  Family labels are non-decreasing in the replica
// index (they start as f_j = j and every resampling copies parents in
// order), so each family is one run of equal labels.  A replica at rank r
// inside its family contributes 2r + 1 to sum_f c_f^2 (the ranks of a
// family of size c give c^2), r + 1 to max_f c_f, and 1 to the number of
// families if r = 0.  The rank needs the family's first index: the last
// start at or before the replica inside the chunk, else (a family that
// began in an earlier chunk) found by binary search for the first label
// equal to the chunk's first.
__global__ void __launch_bounds__(CH_THREADS) k_meas_chunk(const ChunkItem *items, const RunInfo *runs,
                                                           PopState *st)
{
    __shared__ int64_t red[3][CH_THREADS / 64];
    __shared__ int lds_scan[CH_THREADS / 64 + 1];
    __shared__ int first_start;
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rc = S.Rcur;
    const int j0 = it.chunk * CH;
    if (j0 >= Rc) return;
    const int lane = threadIdx.x & 63, wv = wave_id();
    // group partials: groups [j0/64, j0/64 + CH/64), one per lane of wave 0
    int64_t part[MEAS_PART];
#pragma unroll
    for (int k = 0; k < MEAS_PART; ++k) part[k] = 0;
    part[10] = INT32_MAX;
    const int g = j0 / 64 + lane;
    if (wv == 0 && lane < CH / 64 && g * 64 < Rc) {
#pragma unroll
        for (int k = 0; k < MEAS_PART; ++k) part[k] = R.part[it.pop][(size_t)g * MEAS_PART + k];
    }
    // families
    const int32_t *fam = R.fam[it.pop][S.cur];
    if (wv == 0) {
        // first index with the label of replica j0 (labels ascend): a
        // 64-way search by the whole wavefront, the first such index lying
        // in [lo, hi] with fam[hi] equal to the label
        int fs = j0;
        if (j0 > 0 && fam[j0 - 1] == fam[j0]) {
            const int32_t f = fam[j0];
            int lo = 0, hi = j0 - 1;
            while (lo < hi) {
                const int step = (hi - lo + 63) / 64;
                const int p = lo + lane * step;
                const int c = __popcll(__ballot(p < hi && fam[p] < f));   // probes below the first index
                if (c == 0) break;   // fam[lo] is the label
                lo += (c - 1) * step + 1;
                hi = min(hi, lo - 1 + step);
            }
            fs = lo;
        }
        if (lane == 0) first_start = fs;
    }
    const int jb = j0 + threadIdx.x * CH_PER;
    int32_t lab[CH_PER];
    int last = -1;
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        const int j = jb + q;
        lab[q] = j < Rc ? fam[j] : 0;
        if (j < Rc && j > j0 && fam[j - 1] != lab[q]) last = j;
        if (j == j0 && j < Rc && j0 == 0) last = 0;
    }
    // exclusive max-scan of the threads' last starts
    int incl = last;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl = max(incl, t);
    }
    if (lane == 63) lds_scan[wv] = incl;
    __syncthreads();
    int before = first_start;   // start of the family of replica j0
    for (int k = 0; k < wv; ++k) before = max(before, lds_scan[k]);
    {
        const int t = __shfl_up(incl, 1, 64);
        if (lane >= 1) before = max(before, t);
    }
    int64_t sq = 0, mx = 0, nf = 0;
    int s = before;
#pragma unroll
    for (int q = 0; q < CH_PER; ++q) {
        const int j = jb + q;
        if (j < Rc) {
            const bool start = j == 0 || fam[j - 1] != lab[q];
            if (start) s = j;
            const int64_t r = j - s;
            sq += 2 * r + 1;
            mx = r + 1 > mx ? r + 1 : mx;
            nf += start ? 1 : 0;
        }
    }
    sq = wave_sum<int64_t>(sq);
    nf = wave_sum<int64_t>(nf);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) part[k] = wave_sum<int64_t>(part[k]);
        part[10] = wave_min((int)part[10]);
    }
    if (lane == 0) {
        red[0][wv] = sq;
        red[1][wv] = mx;
        red[2][wv] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0, b = 0, c = 0;
        for (int k = 0; k < CH_THREADS / 64; ++k) {
            a += red[0][k];
            b = red[1][k] > b ? red[1][k] : b;
            c += red[2][k];
        }
        unsigned long long *acc = (unsigned long long *)S.acc;
        atomicAdd(&acc[A_FAMSQ], (unsigned long long)a);
        atomicMax(&acc[A_FAMMAX], (unsigned long long)b);
        atomicAdd(&acc[A_NFAM], (unsigned long long)c);
        atomicAdd(&acc[A_SUME], (unsigned long long)part[0]);
        atomicAdd(&acc[A_SUME2], (unsigned long long)part[1]);
        atomicAdd(&acc[A_SUMABSM], (unsigned long long)part[2]);
        atomicAdd(&acc[A_SUMM2], (unsigned long long)part[3]);
        if (part[4]) {
            atomicAdd(&acc[A_NPAIRS], (unsigned long long)part[4]);
            atomicAdd(&acc[A_SUMQ], (unsigned long long)part[5]);
            atomicAdd(&acc[A_SUMABSQ], (unsigned long long)part[6]);
            atomicAdd(&acc[A_SUMQ2], (unsigned long long)part[7]);
            atomicAdd(&acc[A_SUMQL], (unsigned long long)part[8]);
            atomicAdd(&acc[A_SUMQL2], (unsigned long long)part[9]);
        }
        atomicMin(&S.EminAcc, (int)part[10]);
    }
}

// Per run: the record of temperature i for each population, and the
// accumulators reset.  With two populations both records carry the pair
// sums.
__global__ void k_finalize(const RunInfo *runs, PopState *st, int n_runs)
{
    const int run = blockIdx.x * blockDim.x + threadIdx.x;
    if (run >= n_runs) return;
    const RunInfo &R = runs[run];
    int64_t pairs[6] = {0, 0, 0, 0, 0, 0};
    for (int p = 0; p < R.npop; ++p) {
        PopState &S = st[run * MAX_POP + p];
        if (!pop_active(S)) continue;
        const int i = S.i;
        pa_obs o;
        o.R_i = S.Rcur;
        o.lnQ = i == 0 ? 0.0 : S.lnQ;
        o.A = S.A;
        o.sumE = S.acc[A_SUME];
        o.sumE2 = S.acc[A_SUME2];
        o.sumAbsM = S.acc[A_SUMABSM];
        o.sumM2 = S.acc[A_SUMM2];
        if (p == 0)
            for (int k = 0; k < 6; ++k) pairs[k] = S.acc[A_NPAIRS + k];
        o.nPairs = pairs[0];
        o.sumQ = pairs[1];
        o.sumAbsQ = pairs[2];
        o.sumQ2 = pairs[3];
        o.sumQl = pairs[4];
        o.sumQl2 = pairs[5];
        o.famSumSq = S.acc[A_FAMSQ];
        o.famMax = S.acc[A_FAMMAX];
        o.nFam = S.acc[A_NFAM];
        o.Emin = S.EminAcc;
        o.status = PA_OK;
        obs_at(R, i, p) = o;
        S.Emin = S.EminAcc;
        for (int k = 0; k < NACC; ++k) S.acc[k] = 0;
        S.EminAcc = INT32_MAX;
    }
}

// ---------------------------------------------------------------- Sec. IV

// Log free-energy weights per run and temperature: simplified
// ln R_i + A_i (Eq. (simpleWeight)) and full ln R_i + sum_{k<=i}
// ln(R_{k-1}/R) + A_i (Eq. (appropriateWeight)); NaN where the record is not
// OK or the temperature is not reached yet.  One workgroup per run, over the
// temperatures a tile at a time: every thread reads its temperature's
// records and takes the logarithms, then one thread adds the ln(R_{k-1}/R)
// terms from LDS in order of k (the same sums as a sequential pass), instead
// of one thread per run walking all K records with a load and a logarithm in
// each step of a dependent chain.
constexpr int SCAN_THREADS = 256;

__global__ void __launch_bounds__(SCAN_THREADS) k_logw(const RunInfo *runs, const pa_obs *obs, int n_runs,
                                                       int npop_ctx, int pop, int kind, int i_done, double *logw)
{
    __shared__ double term[SCAN_THREADS];   // ln(R_{i-1}/R) of the tile's temperatures, then the running sums
    __shared__ double carry;
    const int run = blockIdx.x, t = threadIdx.x;
    const RunInfo &R = runs[run];
    const bool full = (kind & 1) == PA_W_FULL;
    if (t == 0) carry = 0.0;
    for (int base = 0; base < R.K; base += SCAN_THREADS) {
        const int i = base + t;
        double a = NAN;   // ln R_i + A_i
        if (i < R.K) {
            const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
            term[t] = i > 0 ? log((double)obs[((size_t)(i - 1) * n_runs + run) * npop_ctx + pop].R_i /
                                  (double)R.R)
                            : 0.0;
            if (i <= i_done && o.status == PA_OK && pop < R.npop) a = log((double)o.R_i) + o.A;
        }
        __syncthreads();
        if (t == 0) {
            double cum = carry;
            const int n = min(SCAN_THREADS, R.K - base);
            for (int k = 0; k < n; ++k) {
                if (base + k > 0) cum += term[k];
                term[k] = cum;
            }
            carry = cum;
        }
        __syncthreads();
        if (i < R.K) logw[(size_t)run * R.K + i] = a + (full ? term[t] : 0.0);
        __syncthreads();   // the next tile rewrites term
    }
}

// One thread per (group of M runs, temperature i): weights w = softmax of
// the log weights over the included runs; configurational averages; the
// weighted variance estimators through the Eq. (Wvar_bound) identity; the
// sample variance of w and its log-normal prediction; and ln W[Q_i] with
// the weights of temperature i-1 renormalised over the runs included at i
// (stored in minus_beta_WF, summed over i by k_wavg_cumsum).
__global__ void k_wavg(const RunInfo *runs, const pa_obs *obs, const double *logw, const double *qw, int n_runs,
                       int npop_ctx, int pop, int M, int K, pa_wavg *out)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    const int ngroups = n_runs / M;
    if (gi >= ngroups * K) return;
    const int grp = gi / K, i = gi - grp * K;
    const int N = runs[grp * M].N;
    const double b = runs[grp * M].beta[i];
    pa_wavg w = {};
    double amax = -INFINITY;
    int n = 0;
    for (int m = 0; m < M; ++m) {
        const double a = logw[(size_t)(grp * M + m) * K + i];
        if (!isnan(a)) {
            amax = fmax(amax, a);
            ++n;
        }
    }
    w.n_included = n;
    if (n == 0) {
        const double nan = NAN;
        w.W_e = w.W_e2 = w.Wvar_c = w.Wconf_c = w.W_m = w.W_m2 = nan;
        w.Wvar_chi = w.Wconf_chi = w.W_absq = w.W_q2 = w.W_ql = nan;
        w.minus_beta_WF = w.var_w = w.var_w_pred = nan;
        out[(size_t)grp * K + i] = w;
        return;
    }
    double Z = 0.0;
    for (int m = 0; m < M; ++m) {
        const double a = logw[(size_t)(grp * M + m) * K + i];
        if (!isnan(a)) Z += exp(a - amax);
    }
    const double dN = (double)N;
    double sumA = 0.0;
    for (int m = 0; m < M; ++m) {
        const int run = grp * M + m;
        const double a = logw[(size_t)run * K + i];
        if (isnan(a)) continue;
        const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
        const double wm = exp(a - amax) / Z;
        const double Ri = (double)o.R_i;
        const __int128 vE = (__int128)o.R_i * o.sumE2 - (__int128)o.sumE * o.sumE;
        const __int128 vM = (__int128)o.R_i * o.sumM2 - (__int128)o.sumAbsM * o.sumAbsM;
        w.W_e += wm * ((double)o.sumE / (dN * Ri));
        w.W_e2 += wm * ((double)o.sumE2 / (dN * dN * Ri));
        w.Wconf_c += wm * (b * b * (double)vE / (dN * Ri * Ri));
        w.W_m += wm * ((double)o.sumAbsM / (dN * Ri));
        w.W_m2 += wm * ((double)o.sumM2 / (dN * dN * Ri));
        w.Wconf_chi += wm * (b * (double)vM / (dN * Ri * Ri));
        const double wq = qw[(size_t)run * K + i];   // overlap weights (exclusion applied)
        if (o.nPairs > 0 && !isnan(wq)) {
            const double np = (double)o.nPairs;
            w.W_absq += wq * ((double)o.sumAbsQ / (dN * np));
            w.W_q2 += wq * ((double)o.sumQ2 / (dN * dN * np));
            w.W_ql += wq * ((double)o.sumQl / (2.0 * dN * np));
        }
        sumA += o.A;
    }
    if (isnan(qw[(size_t)(grp * M) * K + i])) w.W_absq = w.W_q2 = w.W_ql = NAN;
    const double meanA = sumA / n;
    double se = 0.0, sm = 0.0, vw = 0.0, va = 0.0;
    for (int m = 0; m < M; ++m) {
        const int run = grp * M + m;
        const double a = logw[(size_t)run * K + i];
        if (isnan(a)) continue;
        const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
        const double wm = exp(a - amax) / Z;
        const double Ri = (double)o.R_i;
        const double e = (double)o.sumE / (dN * Ri), mm = (double)o.sumAbsM / (dN * Ri);
        se += wm * (e - w.W_e) * (e - w.W_e);
        sm += wm * (mm - w.W_m) * (mm - w.W_m);
        vw += (wm - 1.0 / n) * (wm - 1.0 / n);
        va += (o.A - meanA) * (o.A - meanA);
    }
    w.Wvar_c = w.Wconf_c + b * b * dN * se;
    w.Wvar_chi = w.Wconf_chi + b * dN * sm;
    w.var_w = vw / n;
    w.var_w_pred = (exp(va / n) - 1.0) / ((double)n * n);
    if (i == 0) {
        w.minus_beta_WF = NAN;
        for (int m = 0; m < M; ++m) {
            const int run = grp * M + m;
            if (!isnan(logw[(size_t)run * K])) {
                w.minus_beta_WF = obs[((size_t)0 * n_runs + run) * npop_ctx + pop].A;
                break;
            }
        }
    } else {
        double mx = -INFINITY, mx0 = -INFINITY;
        for (int m = 0; m < M; ++m) {
            const int run = grp * M + m;
            if (isnan(logw[(size_t)run * K + i])) continue;
            const double ap = logw[(size_t)run * K + i - 1];
            const double lq = obs[((size_t)i * n_runs + run) * npop_ctx + pop].lnQ;
            mx = fmax(mx, ap + lq);
            mx0 = fmax(mx0, ap);
        }
        double s1 = 0.0, s0 = 0.0;
        for (int m = 0; m < M; ++m) {
            const int run = grp * M + m;
            if (isnan(logw[(size_t)run * K + i])) continue;
            const double ap = logw[(size_t)run * K + i - 1];
            const double lq = obs[((size_t)i * n_runs + run) * npop_ctx + pop].lnQ;
            s1 += exp(ap + lq - mx);
            s0 += exp(ap - mx0);
        }
        w.minus_beta_WF = (mx + log(s1)) - (mx0 + log(s0));
    }
    out[(size_t)grp * K + i] = w;
}

// A family holds more than R_i / 2 replicas in run `run` at temperature i
// (population pop, or either population of a two-population run).
__device__ __forceinline__ bool large_family(const RunInfo &R, const pa_obs *obs, int i, int run, int n_runs,
                                             int npop_ctx, int pop)
{
    for (int p = 0; p < R.npop; ++p) {
        if (p != pop && R.overlap != PA_Q_TWO_POP) continue;
        const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + p];
        if (2 * o.famMax > o.R_i) return true;
    }
    return false;
}

// Weights of the overlap averages: the free-energy weights of k_logw,
// normalised over the included runs of the group (with
// PA_W_EXCLUDE_LARGE_FAMILY also leaving out runs with a family above
// R_i / 2); 0 for a run left out, NaN for every run if none is left.
__global__ void k_qweights(const RunInfo *runs, const pa_obs *obs, const double *logw, int n_runs, int npop_ctx,
                           int pop, int M, int K, int flags, double *qw)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    const int ngroups = n_runs / M;
    if (gi >= ngroups * K) return;
    const int grp = gi / K, i = gi - grp * K;
    const bool excl = flags & PA_W_EXCLUDE_LARGE_FAMILY;
    double amax = -INFINITY;
    int n = 0;
    for (int m = 0; m < M; ++m) {
        const int run = grp * M + m;
        const double a = logw[(size_t)run * K + i];
        if (isnan(a) || (excl && large_family(runs[run], obs, i, run, n_runs, npop_ctx, pop))) continue;
        amax = fmax(amax, a);
        ++n;
    }
    double Z = 0.0;
    for (int m = 0; m < M; ++m) {
        const int run = grp * M + m;
        const double a = logw[(size_t)run * K + i];
        if (isnan(a) || (excl && large_family(runs[run], obs, i, run, n_runs, npop_ctx, pop))) continue;
        Z += exp(a - amax);
    }
    for (int m = 0; m < M; ++m) {
        const int run = grp * M + m;
        const double a = logw[(size_t)run * K + i];
        double w = 0.0;
        if (n == 0) w = NAN;
        else if (!isnan(a) && !(excl && large_family(runs[run], obs, i, run, n_runs, npop_ctx, pop)))
            w = exp(a - amax) / Z;
        qw[(size_t)run * K + i] = w;
    }
}

// Eq. (W_conf_q): one workgroup per (group, temperature), threads over the
// N + 1 bins: W[P(q)](d) = sum_m w_m h_m(d) / nPairs_m, runs in group order.
__global__ void k_wqhist(const RunInfo *runs, const pa_obs *obs, const double *qw, int n_runs, int npop_ctx,
                         int pop, int M, int K, double *out)
{
    const int grp = blockIdx.x / K, i = blockIdx.x - grp * K;
    const int N = runs[grp * M].N;
    const size_t Np1 = (size_t)N + 1;
    double *o = out + ((size_t)grp * K + i) * Np1;
    for (size_t d = threadIdx.x; d < Np1; d += blockDim.x) {
        double acc = 0.0;
        bool none = false;
        for (int m = 0; m < M; ++m) {
            const int run = grp * M + m;
            const double w = qw[(size_t)run * K + i];
            if (isnan(w)) {
                none = true;
                break;
            }
            if (w == 0.0) continue;
            const pa_obs &ob = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
            if (ob.nPairs <= 0) continue;
            const int32_t h = runs[run].qh[((size_t)pop * K + i) * Np1 + d];
            acc += w * ((double)h / (double)ob.nPairs);
        }
        o[d] = none ? NAN : acc;
    }
}

// Family statistics of every (run, temperature) of population pop.
__global__ void k_famstats(const RunInfo *runs, const pa_obs *obs, int n_runs, int npop_ctx, int pop, int K,
                           int i_done, pa_famstat *out)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n_runs * K) return;
    const int run = gi / K, i = gi - run * K;
    const RunInfo &R = runs[run];
    pa_famstat f;
    f.rho_t = NAN;
    f.R_i = 0;
    f.famMax = 0;
    f.large = 0;
    f.excluded = 1;
    if (pop < R.npop && i < R.K && i <= i_done) {
        const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
        f.R_i = (int32_t)o.R_i;
        f.famMax = (int32_t)o.famMax;
        if (o.status == PA_OK && o.R_i > 0) {
            f.rho_t = (double)o.famSumSq / (double)o.R_i;
            f.large = 2 * o.famMax > o.R_i ? 1 : 0;
            f.excluded = large_family(R, obs, i, run, n_runs, npop_ctx, pop) ? 1 : 0;
        }
    }
    out[gi] = f;
}

// -beta_i W[F_i] = ln Z(beta_0) + sum_{k=1..i} ln W[Q_k], Eq. (W_F); NaN
// from the first temperature with no run included on.  One workgroup per
// group of runs: the tile's terms are staged in LDS by all threads and
// summed in order of i by one thread.
__global__ void __launch_bounds__(SCAN_THREADS) k_wavg_cumsum(pa_wavg *out, int ngroups, int K)
{
    __shared__ double v[SCAN_THREADS];
    __shared__ uint8_t none[SCAN_THREADS];   // no run included at that temperature
    __shared__ double carry;
    const int grp = blockIdx.x, t = threadIdx.x;
    if (grp >= ngroups) return;
    if (t == 0) carry = 0.0;
    for (int base = 0; base < K; base += SCAN_THREADS) {
        const int i = base + t;
        if (i < K) {
            const pa_wavg &w = out[(size_t)grp * K + i];
            v[t] = w.minus_beta_WF;
            none[t] = w.n_included == 0;
        }
        __syncthreads();
        if (t == 0) {
            double c = carry;
            const int n = min(SCAN_THREADS, K - base);
            for (int k = 0; k < n; ++k) {
                if (none[k]) c = NAN;
                else c = base + k == 0 ? v[k] : c + v[k];
                v[k] = c;
            }
            carry = c;
        }
        __syncthreads();
        if (i < K) out[(size_t)grp * K + i].minus_beta_WF = v[t];
        __syncthreads();   // the next tile rewrites v and none
    }
}

// ------------------------------------------------------------- launchers

#define PA_CHECK_LAUNCH()                          \
    do {                                           \
        hipError_t e_ = hipGetLastError();         \
        if (e_ != hipSuccess) return e_;           \
    } while (0)

hipError_t launch_fill_u32(void *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    k_fill_u32<<<blocks, 256, 0, s>>>((uint32_t *)p, v, n);
    return hipGetLastError();
}

hipError_t launch_init(const LaunchCtx &c, const uint64_t *dseed)
{
    k_init_couplings<<<c.n_runs, 256, 0, c.stream>>>(c.runs + c.run0, dseed);
    PA_CHECK_LAUNCH();
    k_init_fam<<<c.n_runs, 256, 0, c.stream>>>(c.runs + c.run0);
    PA_CHECK_LAUNCH();
    if (c.repr == PA_MSC64) k_init_spins<PA_MSC64><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs);
    else k_init_spins<PA_INT8><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs);
    return hipGetLastError();
}

hipError_t launch_anneal(const LaunchCtx &c)
{
    k_rw_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    k_rw_finish<<<dim3(c.n_runs, c.npop_ctx), 256, 0, c.stream>>>(c.runs + c.run0,
                                                                 c.st + (size_t)c.run0 * MAX_POP);
    return hipGetLastError();
}

hipError_t launch_resample(const LaunchCtx &c)
{
    k_cnt_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    if (c.any_multinomial) {
        k_mn_draws<<<c.n_chunk_items * c.mn_split, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st,
                                                                              c.mn_split);
        PA_CHECK_LAUNCH();
        k_cnt_scan_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
    }
    k_cnt_finish<<<dim3(c.n_runs, c.npop_ctx), 256, 0, c.stream>>>(c.runs + c.run0,
                                                                  c.st + (size_t)c.run0 * MAX_POP);
    PA_CHECK_LAUNCH();
    k_parent<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    if (c.n_meas_items > 0) {
        const int split = c.copy_split > 1 ? c.copy_split : 1;
        if (c.repr == PA_MSC64)
            k_copy<PA_MSC64><<<c.n_meas_items * split, MEAS_THREADS, 0, c.stream>>>(c.meas_items, c.runs, c.st,
                                                                                  split);
        else
            k_copy<PA_INT8><<<c.n_meas_items * split, MEAS_THREADS, 0, c.stream>>>(c.meas_items, c.runs, c.st,
                                                                                 split);
    }
    return hipGetLastError();
}


// Threads per workgroup of the plain sweep: 256, or 1024 when three rows of
// a very large lattice would not fit in 256 threads' chunks.
int int8_threads(int L) { return 3 * L * 4 <= 256 * I8_CMAX ? 256 : 1024; }

int int8_tile_rows(int L) { return int8_rows_for(L, int8_threads(L)); }

hipError_t launch_sweep_int8_run(const LaunchCtx &c, int run, int L, int groups_cap, int npop, int theta)
{
    const int T = int8_tile_rows(L);
    const int ntiles = (L + T - 1) / T;
    const int nrow = T == L ? L : T + 2;
    const int threads = int8_threads(L);
    const size_t lds = (size_t)nrow * L * 8 + (size_t)T * (L / 2) * 8;
    for (int s = 0; s < theta; ++s)
        for (int colour = 0; colour < 2; ++colour)
            for (int p = 0; p < npop; ++p) {
                if (threads == 256)
                    k_sweep_int8<256><<<groups_cap * ntiles, threads, lds, c.stream>>>(c.runs, c.st, run, p, s,
                                                                                       colour, T, ntiles, c.stats);
                else
                    k_sweep_int8<1024><<<groups_cap * ntiles, threads, lds, c.stream>>>(c.runs, c.st, run, p, s,
                                                                                        colour, T, ntiles, c.stats);
                PA_CHECK_LAUNCH();
            }
    return hipSuccess;
}

size_t msc_lds_bytes(int N, int groups, bool ea, int threads, int mode)
{
    return msc_lds_need(N, groups, ea, threads / 64, mode);
}

// The sweep kernel for a launch: one compiled for a single (L, model) when
// every run of the context has it, else the one that dispatches per item.
using SweepKernel = void (*)(const SweepItem *, int, const RunInfo *, const PopState *, int, unsigned long long *,
                             unsigned int *, unsigned int *, uint32_t);

SweepKernel msc_kernel(int L, int ea)
{
    switch (2 * L + (ea ? 1 : 0)) {
    case 16: return k_sweep_msc<8, false>;
    case 17: return k_sweep_msc<8, true>;
    case 32: return k_sweep_msc<16, false>;
    case 33: return k_sweep_msc<16, true>;
    case 48: return k_sweep_msc<24, false>;
    case 49: return k_sweep_msc<24, true>;
    case 64: return k_sweep_msc<32, false>;
    case 65: return k_sweep_msc<32, true>;
    case 96: return k_sweep_msc<48, false>;
    case 97: return k_sweep_msc<48, true>;
    case 128: return k_sweep_msc<64, false>;
    case 129: return k_sweep_msc<64, true>;
    default: return k_sweep_msc<-1, false>;
    }
}

bool msc_specialised(int L) { return L == 8 || L == 16 || L == 24 || L == 32 || L == 48 || L == 64; }

hipError_t prepare_msc_lds(size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    static const int Ls[] = {8, 16, 24, 32, 48, 64, 0};
    for (int L : Ls)
        for (int ea = 0; ea < 2; ++ea) {
            const hipError_t e = hipFuncSetAttribute((const void *)msc_kernel(L, ea),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// One launch per class (sweep_classes below): the kernel compiled for the
// lattice size and model when every sweeping run shares them; one such
// kernel per (size, model) when every class is large enough to fill the
// chip; else the kernel that dispatches per item.  (On the serving mix,
// whose per-size launches are too small to fill the chip, launching each
// size on its own measured 3.03 against 3.54 thousand flips/ns while busy.)
hipError_t launch_sweep_msc(const LaunchCtx &c)
{
    for (int k = 0; k < c.n_sweep_classes; ++k) {
        const SweepClass &q = c.sweep_cls[k];
        if (q.count == 0) continue;
        const bool persistent = q.grid > 0 && q.grid < q.count;
        // chunked items wait on one another, which only the ticket order of
        // the persistent grid makes safe
        if (q.nchunk > 1 && !persistent) return hipErrorInvalidConfiguration;
        const int grid = persistent ? q.grid : q.count;
        const int mode = c.sweep_dense | (c.sweep_pooled << 8) | (q.L > 0 ? 0 : MSC_WHOLE_LISTS);
        msc_kernel(q.L, q.ea)<<<grid, c.sweep_threads, q.lds, c.stream>>>(
            c.sweep_items + q.first, q.count, c.runs, c.st, mode, c.stats,
            persistent ? c.sweep_queue : nullptr, c.sweep_flags, (uint32_t)q.lds);
        PA_CHECK_LAUNCH();
    }
    return hipSuccess;
}

int sweep_classes(std::vector<SweepItem> &items, const std::vector<int> &run_L, const std::vector<int> &run_ea,
                  SweepClass *cls, int threads, int mode, bool split_ok)
{
    // items of runs without Metropolis sweeps are not launched at all (the
    // kernel of another size must never see them)
    std::vector<SweepItem> out;
    out.reserve(items.size());
    std::vector<int> keys;   // per kept item: 2 L + ea, 0 if L has no kernel of its own
    for (const SweepItem &it : items) {
        const int L = run_L[it.run];
        if (L == 0) continue;
        keys.push_back(msc_specialised(L) ? 2 * L + (run_ea[it.run] ? 1 : 0) : 0);
        out.push_back(it);
    }
    items.swap(out);
    if (items.empty()) return 0;
    auto lds_of = [&](const SweepItem &it, int cmode) {
        const int L = run_L[it.run];
        return msc_lds_bytes(L * L, it.ngroups, run_ea[it.run] != 0, threads, cmode);
    };
    // One launch per (size, model) when every item has a kernel compiled
    // for its size and each class fills at least half of the workgroups
    // that kernel keeps resident: those kernels use fewer registers and the
    // queue rings, so they run more workgroups per CU than the dispatching
    // kernel (the 4096-run batch of four sizes: 6.00 against 6.63 ms per
    // sweep).  Small classes (a serving mix) keep one dispatching launch,
    // since launches that cannot fill the chip one after another are slower.
    std::vector<int> ks(keys);
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    bool split = split_ok && ks.size() > 1 && (int)ks.size() <= MAX_SWEEP_CLASSES && ks[0] != 0;
    std::vector<SweepClass> cand(ks.size());
    for (size_t q = 0; split && q < ks.size(); ++q) {
        SweepClass &C = cand[q];
        C.L = ks[q] / 2;
        C.ea = ks[q] & 1;
        C.count = 0;
        C.lds = 0;
        C.grid = 0;
        for (size_t t = 0; t < items.size(); ++t)
            if (keys[t] == ks[q]) {
                ++C.count;
                C.lds = std::max(C.lds, lds_of(items[t], mode));
            }
        const int resident = sweep_msc_resident(threads, C.lds, C.L, C.ea);
        if (resident <= 0 || 2 * C.count < resident) split = false;
    }
    if (split) {
        // the items of each class together, in their largest-first order
        std::vector<SweepItem> sorted;
        sorted.reserve(items.size());
        for (size_t q = 0; q < ks.size(); ++q) {
            cand[q].first = (int)sorted.size();
            for (size_t t = 0; t < items.size(); ++t)
                if (keys[t] == ks[q]) sorted.push_back(items[t]);
            cls[q] = cand[q];
        }
        items.swap(sorted);
        return (int)ks.size();
    }
    const int key = ks.size() == 1 ? ks[0] : 0;
    SweepClass &C = cls[0];
    C.first = 0;
    C.count = (int)items.size();
    C.L = key / 2;
    C.ea = key & 1;
    C.grid = 0;
    C.lds = 0;
    const int cmode = C.L > 0 ? mode : mode | MSC_WHOLE_LISTS;
    for (const SweepItem &it : items) C.lds = std::max(C.lds, lds_of(it, cmode));
    return 1;
}

int sweep_chunks_auto(int n, int slots)
{
    // makespan in units of one whole item when every item takes the same
    // time: ceil(n K / slots) rounds of 1/K each, plus a cost per extra
    // chunk (loading and storing the lattices once more, a wait on the
    // previous chunk, the chunk's own partial last rounds), measured at
    // about a fifth of an item at L = 64 with three workgroups per CU
    if (slots <= 0 || n <= slots) return 1;
    int best = 1;
    double best_t = 1e300;
    for (int K = 1; K <= MAX_SWEEP_CHUNKS; ++K) {
        const double t = (double)((n * (long)K + slots - 1) / slots) / K + 0.2 * (K - 1);
        if (t < best_t - 1e-9) {
            best_t = t;
            best = K;
        }
    }
    return best;
}

// Makespan, in sweeps, of n equal items of theta sweeps each cut into two
// chunks of a and theta - a sweeps on S workgroups that take tickets in list
// order (every first chunk before any second one); a chunk costs its sweeps
// plus `over` (loading and storing its lattices), and a second chunk starts
// no earlier than its first one ends.
static double two_chunk_makespan(int n, int S, int theta, int a, double over)
{
    std::priority_queue<double, std::vector<double>, std::greater<double>> idle;
    for (int w = 0; w < S; ++w) idle.push(0.0);
    std::vector<double> first_end((size_t)n);
    double end = 0.0;
    for (int lvl = 0; lvl < 2; ++lvl)
        for (int b = 0; b < n; ++b) {
            const double t = idle.top();
            idle.pop();
            const double start = lvl ? std::max(t, first_end[b]) : t;
            const double fin = start + (lvl ? theta - a : a) + over;
            if (!lvl) first_end[b] = fin;
            end = std::max(end, fin);
            idle.push(fin);
        }
    return end;
}

int expand_sweep_chunks(std::vector<SweepItem> &items, SweepClass &cls, int K, const std::vector<int> &run_theta)
{
    cls.nchunk = 1;
    if (K <= 1 || cls.count == 0) return 0;
    if (K > MAX_SWEEP_CHUNKS || cls.first != 0 || cls.count != (int)items.size()) return -1;
    const int n = cls.count;
    // Two chunks: the cut that the makespan above, at the largest theta of
    // the list and about 0.6 sweeps per chunk, says ends the launch first
    // (the first chunk at least half; the even cut on ties).  At L = 64,
    // R = 1e5 (1563 items, 768 workgroups) that is 7 and 3 sweeps, measured
    // 1.3 % faster than 5 and 5; for the two populations at L = 32 (3125
    // items, 1280 workgroups) it is 5 and 5, where 8 and 2 measured 5 %
    // slower.  More chunks: as even as possible, the larger first.
    int theta_ref = 0;
    for (const SweepItem &it : items) theta_ref = std::max(theta_ref, run_theta[it.run]);
    int cut_ref = (theta_ref + 1) / 2;
    if (K == 2 && theta_ref >= 2 && cls.grid > 0) {
        double best = two_chunk_makespan(n, cls.grid, theta_ref, cut_ref, 0.6);
        for (int a = cut_ref + 1; a < theta_ref; ++a) {
            const double t = two_chunk_makespan(n, cls.grid, theta_ref, a, 0.6);
            if (t < best - 1e-9) {
                best = t;
                cut_ref = a;
            }
        }
    }
    std::vector<SweepItem> out((size_t)n * K);
    for (int c = 0; c < K; ++c)
        for (int b = 0; b < n; ++b) {
            SweepItem it = items[b];
            const long theta = run_theta[it.run];
            it.chunk = c;
            it.nchunk = K;
            it.base = b;
            it.cut = theta_ref > 0 ? (int)((theta * cut_ref + theta_ref / 2) / theta_ref) : 0;
            out[(size_t)c * n + b] = it;
        }
    items.swap(out);
    cls.count = n * K;
    cls.nchunk = K;
    return 0;
}

bool sweep_class_grids(SweepClass *cls, int n, int threads, bool persistent)
{
    for (int k = 0; k < n; ++k) {
        cls[k].grid = 0;
        if (!persistent) continue;
        const int resident = sweep_msc_resident(threads, cls[k].lds, cls[k].L, cls[k].ea);
        if (resident <= 0) return false;
        cls[k].grid = resident;
    }
    return true;
}

int sweep_msc_resident(int threads, size_t lds, int L, int ea)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, msc_kernel(L, ea), threads, lds) != hipSuccess)
        return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_dos_sample(const LaunchCtx &c)
{
    if (!c.any_exact_dos || c.n_items == 0) return hipSuccess;
    k_dos_sample<<<(c.n_items + 3) / 4, 256, 0, c.stream>>>(c.items, c.n_items, c.runs, c.st);
    return hipGetLastError();
}

hipError_t launch_measure(const LaunchCtx &c)
{
    if (c.any_wang && c.n_runs > 0) {
        k_wang_pairs<<<c.n_runs, WANG_THREADS, sizeof(int32_t) * (size_t)c.wang_lds_ints, c.stream>>>(
            c.runs, c.st, c.run0, c.wang_lds_ints);
        PA_CHECK_LAUNCH();
        const int blocks = (c.n_items + 3) / 4;
        if (c.repr == PA_INT8)
            k_wang_rows<PA_INT8><<<blocks, 256, 0, c.stream>>>(c.items, c.n_items, c.runs, c.st);
        else
            k_wang_rows<PA_MSC64><<<blocks, 256, 0, c.stream>>>(c.items, c.n_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
        k_wang_gather<<<blocks, 256, 0, c.stream>>>(c.items, c.n_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
    }
    if (c.n_meas_items > 0) {
        // the variant without overlap counters when no run measures overlaps
        // (fewer registers live in the site loop)
        if (c.repr == PA_MSC64 && c.any_overlap)
            k_measure<PA_MSC64, true><<<c.n_meas_items, MEAS_THREADS, 0, c.stream>>>(c.meas_items, c.runs, c.st);
        else if (c.repr == PA_MSC64)
            k_measure<PA_MSC64, false><<<c.n_meas_items, MEAS_THREADS, 0, c.stream>>>(c.meas_items, c.runs, c.st);
        else if (c.any_overlap)
            k_measure<PA_INT8, true><<<c.n_meas_items, MEAS_THREADS, MEAS_STAGE_BYTES, c.stream>>>(c.meas_items, c.runs, c.st);
        else
            k_measure<PA_INT8, false><<<c.n_meas_items, MEAS_THREADS, MEAS_STAGE_BYTES, c.stream>>>(c.meas_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
    }
    k_meas_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    k_finalize<<<(c.n_runs + 63) / 64, 64, 0, c.stream>>>(c.runs + c.run0, c.st + (size_t)c.run0 * MAX_POP,
                                                          c.n_runs);
    return hipGetLastError();
}

hipError_t launch_qweights(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K, int i_done,
                           double *logw, double *qw)
{
    k_logw<<<c.n_runs, SCAN_THREADS, 0, c.stream>>>(c.runs, obs, c.n_runs, c.npop_ctx, pop, kind, i_done, logw);
    PA_CHECK_LAUNCH();
    const int ng = c.n_runs / M;
    k_qweights<<<(ng * K + 127) / 128, 128, 0, c.stream>>>(c.runs, obs, logw, c.n_runs, c.npop_ctx, pop, M, K,
                                                          kind & ~1, qw);
    return hipGetLastError();
}

hipError_t launch_wqhist(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K, int i_done,
                         double *logw, double *qw, double *out)
{
    if (launch_qweights(c, obs, M, kind, pop, K, i_done, logw, qw) != hipSuccess) return hipGetLastError();
    const int ng = c.n_runs / M;
    k_wqhist<<<ng * K, 256, 0, c.stream>>>(c.runs, obs, qw, c.n_runs, c.npop_ctx, pop, M, K, out);
    return hipGetLastError();
}

hipError_t launch_famstats(const LaunchCtx &c, const pa_obs *obs, int pop, int K, int i_done, pa_famstat *out)
{
    k_famstats<<<(c.n_runs * K + 255) / 256, 256, 0, c.stream>>>(c.runs, obs, c.n_runs, c.npop_ctx, pop, K,
                                                                 i_done, out);
    return hipGetLastError();
}

hipError_t launch_wavg(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K,
                       int i_done, double *logw, double *qw, pa_wavg *out)
{
    if (launch_qweights(c, obs, M, kind, pop, K, i_done, logw, qw) != hipSuccess) return hipGetLastError();
    const int ng = c.n_runs / M;
    k_wavg<<<(ng * K + 127) / 128, 128, 0, c.stream>>>(c.runs, obs, logw, qw, c.n_runs, c.npop_ctx, pop, M, K,
                                                      out);
    PA_CHECK_LAUNCH();
    k_wavg_cumsum<<<ng, SCAN_THREADS, 0, c.stream>>>(out, ng, K);
    return hipGetLastError();
}

}  // namespace pa
