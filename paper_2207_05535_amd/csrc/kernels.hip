// kernels.hip -- HIP kernels of the population-annealing temperature step
// for gfx950 (CDNA4, 64-wide wavefronts).
//
// Step (i)   k_init_couplings, k_init_spins           (Sec. II B, III A)
// Step (ii)  k_rw_chunk, k_rw_finish                   (Eqs. (QBoltz), (F))
// Step (iii) k_cnt_chunk, k_mn_draws, k_cnt_scan_chunk, k_cnt_finish,
//            k_parent, k_copy                          (Sec. II B, IV D, V A 1)
// Step (iv)  k_sweep_int8 (one colour of one run per launch),
//            k_sweep_msc (all runs, lattice in LDS for all theta sweeps)
// Step (v)   k_measure, k_finalize                     (Eqs. (e)-(chi), Sec. III D)
// Sec. IV    k_logw, k_wavg, k_wavg_cumsum
//
// Population-wide reductions and scans are split into fixed-size chunks of
// CH replicas (one workgroup each) plus a single-workgroup pass over the
// chunk totals, so every result is independent of the launch shape and the
// floating-point sums have one fixed order.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "launch.hpp"
#include "metropolis.hpp"
#include "pa_internal.hpp"
#include "philox.hpp"

namespace pa {

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

// Exclusive scan of one value per thread across a workgroup of BS threads
// (BS a multiple of 64); returns the exclusive prefix, *total the sum.
template <typename T, int BS>
__device__ __forceinline__ T block_exscan(T v, T *lds, T *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
            uint4 v[4];
            const uint32_t lo = (uint32_t)plane, hi = (uint32_t)(plane >> 32);
            for (int q = 0; q < 4; ++q) {
                const uint32_t bits = (q < 2 ? lo : hi) >> (16 * (q & 1));
                v[q].x = 0x01010101u ^ negmask4(bits & 15u);
                v[q].y = 0x01010101u ^ negmask4((bits >> 4) & 15u);
                v[q].z = 0x01010101u ^ negmask4((bits >> 8) & 15u);
                v[q].w = 0x01010101u ^ negmask4((bits >> 12) & 15u);
            }
            uint4 *dst = (uint4 *)(R.spins[it.pop][0] + site * 64);
            for (int q = 0; q < 4; ++q) dst[q] = v[q];
        }
    }
}

__global__ void k_init_fam(const RunInfo *runs, int npop_ctx)
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
                                                          const PopState *st, int npop_ctx)
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
__global__ void k_rw_finish(const RunInfo *runs, PopState *st, int npop_ctx)
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
__global__ void __launch_bounds__(CH_THREADS) k_mn_draws(const ChunkItem *items, const RunInfo *runs,
                                                          const PopState *st)
{
    const ChunkItem it = items[blockIdx.x];
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
    for (int q = 0; q < CH_PER; ++q) {
        const int d = d0 + threadIdx.x + q * CH_THREADS;
        if (d >= R.R) break;
        const u32x4 o = philox10((uint32_t)d, 0, (uint32_t)S.i, c3, R.key0, R.key1);
        const uint64_t v = (uint64_t)o.x | ((uint64_t)o.y << 32);
        const uint64_t t = umul64hi(v, SX);
        int lo = 0, hi = Rp - 1;      // largest j with P_j <= t
        while (lo < hi) {
            const int mid = lo + ((hi - lo + 1) >> 1);
            const uint64_t pm = B[mid / CH] + P[mid];
            if (pm <= t) lo = mid;
            else hi = mid - 1;
        }
        atomicAdd(&r[lo], 1);
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

__device__ void freeze_run(const RunInfo &R, PopState &S, int pop, int i, int32_t status,
                           int n_runs, int npop_ctx)
{
    for (int k = i + threadIdx.x; k < R.K; k += blockDim.x) {
        pa_obs o = {};
        o.status = status;
        R.obs[((size_t)k * n_runs + R.run) * npop_ctx + pop] = o;
    }
    if (threadIdx.x == 0) {
        S.status = status;
        S.moved = 0;
    }
}

// Chunk bases of the count prefix, R_i = sum r_j; capacity and empty-
// population checks (the run is frozen with that status); otherwise the
// new population becomes current: the copy reads buffer src, writes cur.
__global__ void k_cnt_finish(const RunInfo *runs, PopState *st, int n_runs, int npop_ctx)
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
        freeze_run(R, S, pop, S.i, PA_ERR_CAPACITY, n_runs, npop_ctx);
        return;
    }
    if (carry == 0) {
        freeze_run(R, S, pop, S.i, PA_ERR_NUMERIC, n_runs, npop_ctx);
        return;
    }
    if (threadIdx.x == 0) {
        S.src = S.cur;
        S.cur = S.cur ^ 1;
        S.Rcur = (int32_t)carry;
    }
}

// Parent of every child slot c < R_i: the largest j with C_j <= c (then
// r_j > 0), C_j = base32[chunk] + chunk-local prefix.
__global__ void __launch_bounds__(CH_THREADS) k_parent(const ChunkItem *items, const RunInfo *runs,
                                                        const PopState *st)
{
    const ChunkItem it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rc = S.Rcur, Rp = S.Rprev;
    const int c0 = it.chunk * CH;
    if (c0 >= Rc) return;
    const int32_t *C = R.C[it.pop];
    const int32_t *B = R.base32[it.pop];
    int32_t *par = R.parent[it.pop];
    for (int q = 0; q < CH_PER; ++q) {
        const int c = c0 + threadIdx.x + q * CH_THREADS;
        if (c >= Rc) break;
        int lo = 0, hi = Rp - 1;
        while (lo < hi) {
            const int mid = lo + ((hi - lo + 1) >> 1);
            if (B[mid / CH] + C[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        par[c] = lo;
    }
}

// Copy of spins, energies and family labels into the child slots.  One
// wavefront per 64 children (one replica group); int8: lane = child, one
// byte per site; MSC: each child's bit gathered from its parent's word and
// the 64 bits assembled with a wave ballot.
template <int REPR>
__global__ void __launch_bounds__(256) k_copy(const Item *items, const RunInfo *runs, const PopState *st)
{
    const Item it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rc = S.Rcur;
    const int G = it.group;
    if (G * 64 >= Rc) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = G * 64 + lane;
    const bool valid = c < Rc;
    const int p = valid ? R.parent[it.pop][c] : 0;
    const int N = R.N;
    const int per = (N + 3) / 4;
    const int n0 = wv * per, n1 = min(N, n0 + per);
    if (REPR == PA_MSC64) {
        const uint64_t *src = (const uint64_t *)R.spins[it.pop][S.src] + (size_t)(p >> 6) * N;
        uint64_t *dst = (uint64_t *)R.spins[it.pop][S.cur] + (size_t)G * N;
        const int pb = p & 63;
        for (int nb = n0; nb < n1; nb += 64) {
            uint64_t mine = 0;
            const int cnt = min(64, n1 - nb);
            for (int k = 0; k < cnt; ++k) {
                const int bit = valid ? (int)((src[nb + k] >> pb) & 1u) : 0;
                const uint64_t m = __ballot(bit);
                if (lane == k) mine = m;
            }
            if (lane < cnt) dst[nb + lane] = mine;
        }
    } else {
        const uint8_t *src = R.spins[it.pop][S.src] + (size_t)(p >> 6) * N * 64 + (p & 63);
        uint8_t *dst = R.spins[it.pop][S.cur] + (size_t)G * N * 64 + lane;
        for (int n = n0; n < n1; ++n) dst[(size_t)n * 64] = valid ? src[(size_t)n * 64] : (uint8_t)1;
    }
    if (wv == 0 && valid) {
        R.E[it.pop][S.cur][c] = R.E[it.pop][S.src][p];
        R.fam[it.pop][S.cur][c] = R.fam[it.pop][S.src][p];
    }
}

// ------------------------------------------------------------- step (iv)

// One atomic per wavefront: the sweep kernels' exact work counts.
__device__ __forceinline__ void flush_stats(unsigned long long *stats, uint32_t words, uint32_t calls,
                                            uint32_t flips)
{
    const unsigned long long w = wave_sum<unsigned long long>(words);
    const unsigned long long c = wave_sum<unsigned long long>(calls);
    const unsigned long long f = wave_sum<unsigned long long>(flips);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&stats[ST_WORDS], w);
        atomicAdd(&stats[ST_CALLS], c);
        atomicAdd(&stats[ST_FLIPS], f);
    }
}

__device__ __forceinline__ uint64_t jmask(uint8_t b, int bit) { return ((b >> bit) & 1u) ? ~0ull : 0ull; }

// Plain path: one colour of one run per launch, int8 spins.  A workgroup
// takes T rows of one replica group: it stages the other colour's sites of
// rows y0-1 .. y0+T (bit-packed, 8 bytes per site) in LDS, then updates its
// own colour's sites in place in HBM, one site (64 replicas) per thread.
__global__ void __launch_bounds__(256) k_sweep_int8(const RunInfo *runs, const PopState *st, int run,
                                                     int pop, int s, int colour, int T, int ntiles,
                                                     unsigned long long *stats)
{
    extern __shared__ uint64_t nb[];
    const RunInfo &R = runs[run];
    const PopState &S = st[run * MAX_POP + pop];
    if (!pop_active(S)) return;
    const int g = blockIdx.x / ntiles, tile = blockIdx.x % ntiles;
    const int Rc = S.Rcur;
    if (g * 64 >= Rc) return;
    const int L = R.L, N = R.N, half = L >> 1;
    const int y0 = tile * T;
    const int rows = min(T, L - y0);
    const int co = colour ^ 1;
    uint8_t *base = R.spins[pop][S.cur] + (size_t)g * N * 64;
    for (int idx = threadIdx.x; idx < (rows + 2) * half; idx += blockDim.x) {
        const int rr = idx / half, m = idx - rr * half;
        const int y = (y0 - 1 + rr + L) % L;
        const int x = 2 * m + ((y + co) & 1);
        const uint4 *src = (const uint4 *)(base + (size_t)(y * L + x) * 64);
        uint4 v[4] = {src[0], src[1], src[2], src[3]};
        nb[idx] = pack64(v);
    }
    __syncthreads();
    const int i = S.i;
    const Thresholds Th = thresholds_of(R.tabT, i);
    const uint32_t c3 = (TAG_SWEEP << 28) | ((uint32_t)pop << 24) | (uint32_t)s;
    const uint64_t valid = (Rc - g * 64 >= 64) ? ~0ull : ((1ull << (Rc - g * 64)) - 1);
    const uint32_t lanes = (uint32_t)__popcll(valid);
    uint32_t nwords = 0, ncalls = 0;
    for (int idx = threadIdx.x; idx < rows * half; idx += blockDim.x) {
        const int yy = idx / half, m = idx - yy * half;
        const int y = y0 + yy;
        const int x = 2 * m + ((y + colour) & 1);
        const int n = y * L + x;
        const int xr = x + 1 == L ? 0 : x + 1, xl = x == 0 ? L - 1 : x - 1;
        const int yu = y == 0 ? L - 1 : y - 1;
        uint4 *p = (uint4 *)(base + (size_t)n * 64);
        uint4 v[4] = {p[0], p[1], p[2], p[3]};
        const uint64_t w = pack64(v);
        const uint64_t wr = nb[(yy + 1) * half + (xr >> 1)];
        const uint64_t wl = nb[(yy + 1) * half + (xl >> 1)];
        const uint64_t wd = nb[(yy + 2) * half + m];
        const uint64_t wu = nb[yy * half + m];
        const uint8_t jn = R.jbits[n];
        const uint64_t F = flip_mask(w, wr, wl, wd, wu, jmask(jn, 0), jmask(R.jbits[y * L + xl], 0),
                                     jmask(jn, 1), jmask(R.jbits[yu * L + x], 1), Th, valid,
                                     (uint32_t)n, (uint32_t)g, (uint32_t)i, c3, R.key0, R.key1, ncalls);
        ++nwords;
        if (F) {
            apply64(v, F);
            p[0] = v[0];
            p[1] = v[1];
            p[2] = v[2];
            p[3] = v[3];
        }
    }
    flush_stats(stats, nwords, ncalls, nwords * lanes);
}

// Batched path: every (run, pop, group) item of the context in one launch;
// the group's lattice (N words) and couplings stay in LDS for all theta
// sweeps, split by colour so that a colour's sites are contiguous.
__global__ void __launch_bounds__(256) k_sweep_msc(const Item *items, const RunInfo *runs, const PopState *st,
                                                    unsigned long long *stats)
{
    extern __shared__ uint64_t lat[];
    const Item it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    const PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int g = it.group;
    const int Rc = S.Rcur;
    if (g * 64 >= Rc || R.theta == 0) return;
    const int L = R.L, N = R.N, half = L >> 1, nh = N >> 1;
    uint8_t *jb = (uint8_t *)(lat + N);
    uint64_t *base = (uint64_t *)R.spins[it.pop][S.cur] + (size_t)g * N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int y = n / L, x = n - y * L;
        lat[((x + y) & 1) * nh + y * half + (x >> 1)] = base[n];
        jb[n] = R.jbits[n];
    }
    const int i = S.i;
    const Thresholds Th = thresholds_of(R.tabT, i);
    const uint32_t c3p = (TAG_SWEEP << 28) | ((uint32_t)it.pop << 24);
    const uint64_t valid = (Rc - g * 64 >= 64) ? ~0ull : ((1ull << (Rc - g * 64)) - 1);
    const uint32_t lanes = (uint32_t)__popcll(valid);
    uint32_t nwords = 0, ncalls = 0;
    for (int s = 0; s < R.theta; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            __syncthreads();
            uint64_t *own = lat + colour * nh;
            const uint64_t *oth = lat + (colour ^ 1) * nh;
            for (int k = threadIdx.x; k < nh; k += blockDim.x) {
                const int y = k / half, m = k - y * half;
                const int x = 2 * m + ((y + colour) & 1);
                const int n = y * L + x;
                const int xr = x + 1 == L ? 0 : x + 1, xl = x == 0 ? L - 1 : x - 1;
                const int yd = y + 1 == L ? 0 : y + 1, yu = y == 0 ? L - 1 : y - 1;
                const uint64_t w = own[k];
                const uint8_t jn = jb[n];
                const uint64_t F = flip_mask(w, oth[y * half + (xr >> 1)], oth[y * half + (xl >> 1)],
                                             oth[yd * half + m], oth[yu * half + m], jmask(jn, 0),
                                             jmask(jb[y * L + xl], 0), jmask(jn, 1),
                                             jmask(jb[yu * L + x], 1), Th, valid, (uint32_t)n,
                                             (uint32_t)g, (uint32_t)i, c3p | (uint32_t)s, R.key0, R.key1,
                                             ncalls);
                ++nwords;
                own[k] = w ^ F;
            }
        }
    }
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int y = n / L, x = n - y * L;
        base[n] = lat[((x + y) & 1) * nh + y * half + (x >> 1)];
    }
    flush_stats(stats, nwords, ncalls, nwords * lanes);
}

// -------------------------------------------------------------- step (v)

template <int REPR>
__device__ __forceinline__ int spin_bit(const uint8_t *buf, int j, int n, int N)
{
    if (REPR == PA_MSC64)
        return (int)((((const uint64_t *)buf)[(size_t)(j >> 6) * N + n] >> (j & 63)) & 1u);
    return buf[((size_t)(j >> 6) * N + n) * 64 + (j & 63)] >> 7;
}

// Per replica (lane = replica of a 64-group, 4 waves splitting the sites):
// E_j = 2 (#unsatisfied bonds) - 2N, M_j = N - 2 (#down spins); per pair
// the Hamming distance d (Q = N - 2d) and the number of bonds whose product
// differs (Q_l = 2N - 2 d_l).  Integer sums go to the per-population
// accumulators, family sizes to the family histogram.
template <int REPR>
__global__ void __launch_bounds__(256) k_measure(const Item *items, const RunInfo *runs, PopState *st)
{
    __shared__ int red[4][4][64];
    const Item it = items[blockIdx.x];
    const RunInfo &R = runs[it.run];
    PopState &S = st[it.run * MAX_POP + it.pop];
    if (!pop_active(S)) return;
    const int Rc = S.Rcur;
    const int g = it.group;
    if (g * 64 >= Rc) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = g * 64 + lane;
    const bool valid = j < Rc;
    const int L = R.L, N = R.N;
    const uint8_t *buf = R.spins[it.pop][S.cur];
    bool pair = false;
    int pj = 0;
    const uint8_t *pbuf = buf;
    if (R.overlap == PA_Q_INDEX_SHIFT) {
        const int h = Rc >> 1;
        pair = j < h;
        pj = j + h;
    } else if (R.overlap == PA_Q_TWO_POP && it.pop == 0) {
        const PopState &S1 = st[it.run * MAX_POP + 1];
        if (pop_active(S1)) {
            pair = j < min(Rc, S1.Rcur);
            pj = j;
            pbuf = R.spins[1][S1.cur];
        }
    }
    const int jj = valid ? j : g * 64;
    const int pjj = pair ? pj : 0;
    int unsat = 0, down = 0, ham = 0, dl = 0;
    const int per = (N + 3) / 4;
    const int n0 = wv * per, n1 = min(N, n0 + per);
    for (int n = n0; n < n1; ++n) {
        const int y = n / L, x = n - y * L;
        const int nr = y * L + (x + 1 == L ? 0 : x + 1);
        const int nd = (y + 1 == L ? 0 : y + 1) * L + x;
        const int jbn = R.jbits[n];
        const int s = spin_bit<REPR>(buf, jj, n, N);
        const int sr = spin_bit<REPR>(buf, jj, nr, N);
        const int sd = spin_bit<REPR>(buf, jj, nd, N);
        unsat += (s ^ sr ^ (jbn & 1)) + (s ^ sd ^ ((jbn >> 1) & 1));
        down += s;
        if (pair) {
            const int t = spin_bit<REPR>(pbuf, pjj, n, N);
            const int tr = spin_bit<REPR>(pbuf, pjj, nr, N);
            const int td = spin_bit<REPR>(pbuf, pjj, nd, N);
            ham += s ^ t;
            dl += (s ^ sr ^ t ^ tr) + (s ^ sd ^ t ^ td);
        }
    }
    red[0][wv][lane] = unsat;
    red[1][wv][lane] = down;
    red[2][wv][lane] = ham;
    red[3][wv][lane] = dl;
    __syncthreads();
    if (wv != 0) return;
    unsat = red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
    down = red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane];
    ham = red[2][0][lane] + red[2][1][lane] + red[2][2][lane] + red[2][3][lane];
    dl = red[3][0][lane] + red[3][1][lane] + red[3][2][lane] + red[3][3][lane];
    const int64_t E = 2 * unsat - 2 * N;
    const int64_t M = N - 2 * down;
    if (valid) {
        R.E[it.pop][S.cur][j] = (int32_t)E;
        atomicAdd(&R.famcnt[it.pop][R.fam[it.pop][S.cur][j]], 1);
    }
    const int64_t v = valid ? 1 : 0;
    const int64_t sE = wave_sum<int64_t>(v * E);
    const int64_t sE2 = wave_sum<int64_t>(v * E * E);
    const int64_t sM = wave_sum<int64_t>(v * (M < 0 ? -M : M));
    const int64_t sM2 = wave_sum<int64_t>(v * M * M);
    const int emin = wave_min(valid ? (int)E : INT32_MAX);
    const int64_t pv = pair ? 1 : 0;
    const int64_t Q = N - 2 * ham, Ql = 2 * N - 2 * dl;
    const int64_t np = wave_sum<int64_t>(pv);
    const int64_t sQ = wave_sum<int64_t>(pv * Q);
    const int64_t sAQ = wave_sum<int64_t>(pv * (Q < 0 ? -Q : Q));
    const int64_t sQ2 = wave_sum<int64_t>(pv * Q * Q);
    const int64_t sQl = wave_sum<int64_t>(pv * Ql);
    const int64_t sQl2 = wave_sum<int64_t>(pv * Ql * Ql);
    if (pair && R.qhist) {
        const size_t Np1 = (size_t)N + 1;
        atomicAdd(&R.qh[((size_t)it.pop * R.K + S.i) * Np1 + ham], 1);
        if (R.overlap == PA_Q_TWO_POP) atomicAdd(&R.qh[((size_t)1 * R.K + S.i) * Np1 + ham], 1);
    }
    if (lane == 0) {
        unsigned long long *acc = (unsigned long long *)S.acc;
        atomicAdd(&acc[A_SUME], (unsigned long long)sE);
        atomicAdd(&acc[A_SUME2], (unsigned long long)sE2);
        atomicAdd(&acc[A_SUMABSM], (unsigned long long)sM);
        atomicAdd(&acc[A_SUMM2], (unsigned long long)sM2);
        if (np) {
            atomicAdd(&acc[A_NPAIRS], (unsigned long long)np);
            atomicAdd(&acc[A_SUMQ], (unsigned long long)sQ);
            atomicAdd(&acc[A_SUMABSQ], (unsigned long long)sAQ);
            atomicAdd(&acc[A_SUMQ2], (unsigned long long)sQ2);
            atomicAdd(&acc[A_SUMQL], (unsigned long long)sQl);
            atomicAdd(&acc[A_SUMQL2], (unsigned long long)sQl2);
        }
        atomicMin(&S.EminAcc, emin);
    }
}

// Per run: family statistics from the histogram (then cleared), the record
// of temperature i for each population, and the accumulators reset.  With
// two populations both records carry the pair sums.
__global__ void k_finalize(const RunInfo *runs, PopState *st, int n_runs, int npop_ctx)
{
    __shared__ int64_t red[3][256];
    const int run = blockIdx.x;
    const RunInfo &R = runs[run];
    int64_t pairs[6] = {0, 0, 0, 0, 0, 0};
    for (int p = 0; p < R.npop; ++p) {
        PopState &S = st[run * MAX_POP + p];
        if (!pop_active(S)) continue;
        int64_t sq = 0, mx = 0, nz = 0;
        int32_t *fc = R.famcnt[p];
        for (int f = threadIdx.x; f < R.R; f += blockDim.x) {
            const int64_t c = fc[f];
            sq += c * c;
            mx = c > mx ? c : mx;
            nz += c > 0;
            fc[f] = 0;
        }
        red[0][threadIdx.x] = sq;
        red[1][threadIdx.x] = mx;
        red[2][threadIdx.x] = nz;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                red[0][threadIdx.x] += red[0][threadIdx.x + o];
                red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + o]);
                red[2][threadIdx.x] += red[2][threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int i = S.i;
            pa_obs o;
            o.R_i = S.Rcur;
            o.lnQ = i == 0 ? 0.0 : S.lnQ;
            o.A = S.A;
            o.sumE = S.acc[A_SUME];
            o.sumE2 = S.acc[A_SUME2];
            o.sumAbsM = S.acc[A_SUMABSM];
            o.sumM2 = S.acc[A_SUMM2];
            if (p == 0) {
                for (int k = 0; k < 6; ++k) pairs[k] = S.acc[A_NPAIRS + k];
            }
            o.nPairs = pairs[0];
            o.sumQ = pairs[1];
            o.sumAbsQ = pairs[2];
            o.sumQ2 = pairs[3];
            o.sumQl = pairs[4];
            o.sumQl2 = pairs[5];
            o.famSumSq = red[0][0];
            o.famMax = red[1][0];
            o.nFam = red[2][0];
            o.Emin = S.EminAcc;
            o.status = PA_OK;
            R.obs[((size_t)i * n_runs + run) * npop_ctx + p] = o;
            S.Emin = S.EminAcc;
            for (int k = 0; k < NACC; ++k) S.acc[k] = 0;
            S.EminAcc = INT32_MAX;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- Sec. IV

// Log free-energy weights per run and temperature: simplified
// ln R_i + A_i (Eq. (simpleWeight)) and full ln R_i + sum_{k<=i}
// ln(R_{k-1}/R) + A_i (Eq. (appropriateWeight)); NaN where the record is not
// OK or the temperature is not reached yet.
__global__ void k_logw(const RunInfo *runs, const pa_obs *obs, int n_runs, int npop_ctx, int pop,
                       int kind, int i_done, double *logw)
{
    const int run = blockIdx.x * blockDim.x + threadIdx.x;
    if (run >= n_runs) return;
    const RunInfo &R = runs[run];
    double cum = 0.0;
    for (int i = 0; i < R.K; ++i) {
        const pa_obs &o = obs[((size_t)i * n_runs + run) * npop_ctx + pop];
        if (i > 0) {
            const pa_obs &op = obs[((size_t)(i - 1) * n_runs + run) * npop_ctx + pop];
            cum += log((double)op.R_i / (double)R.R);
        }
        double a = NAN;
        if (i <= i_done && o.status == PA_OK && pop < R.npop)
            a = log((double)o.R_i) + o.A + (kind == PA_W_FULL ? cum : 0.0);
        logw[(size_t)run * R.K + i] = a;
    }
}

// One thread per (group of M runs, temperature i): weights w = softmax of
// the log weights over the included runs; configurational averages; the
// weighted variance estimators through the Eq. (Wvar_bound) identity; the
// sample variance of w and its log-normal prediction; and ln W[Q_i] with
// the weights of temperature i-1 renormalised over the runs included at i
// (stored in minus_beta_WF, summed over i by k_wavg_cumsum).
__global__ void k_wavg(const RunInfo *runs, const pa_obs *obs, const double *logw, int n_runs,
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
        if (o.nPairs > 0) {
            const double np = (double)o.nPairs;
            w.W_absq += wm * ((double)o.sumAbsQ / (dN * np));
            w.W_q2 += wm * ((double)o.sumQ2 / (dN * dN * np));
            w.W_ql += wm * ((double)o.sumQl / (2.0 * dN * np));
        }
        sumA += o.A;
    }
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

// -beta_i W[F_i] = ln Z(beta_0) + sum_{k=1..i} ln W[Q_k], Eq. (W_F).
__global__ void k_wavg_cumsum(pa_wavg *out, int ngroups, int K)
{
    const int grp = blockIdx.x * blockDim.x + threadIdx.x;
    if (grp >= ngroups) return;
    double c = 0.0;
    for (int i = 0; i < K; ++i) {
        pa_wavg &w = out[(size_t)grp * K + i];
        if (w.n_included == 0) c = NAN;
        else c = i == 0 ? w.minus_beta_WF : c + w.minus_beta_WF;
        w.minus_beta_WF = c;
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
    k_init_couplings<<<c.n_runs, 256, 0, c.stream>>>(c.runs, dseed);
    PA_CHECK_LAUNCH();
    k_init_fam<<<c.n_runs, 256, 0, c.stream>>>(c.runs, c.npop_ctx);
    PA_CHECK_LAUNCH();
    if (c.repr == PA_MSC64) k_init_spins<PA_MSC64><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs);
    else k_init_spins<PA_INT8><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs);
    return hipGetLastError();
}

hipError_t launch_anneal(const LaunchCtx &c)
{
    k_rw_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st, c.npop_ctx);
    PA_CHECK_LAUNCH();
    k_rw_finish<<<dim3(c.n_runs, c.npop_ctx), 256, 0, c.stream>>>(c.runs, c.st, c.npop_ctx);
    return hipGetLastError();
}

hipError_t launch_resample(const LaunchCtx &c)
{
    k_cnt_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    if (c.any_multinomial) {
        k_mn_draws<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
        k_cnt_scan_chunk<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
        PA_CHECK_LAUNCH();
    }
    k_cnt_finish<<<dim3(c.n_runs, c.npop_ctx), 256, 0, c.stream>>>(c.runs, c.st, c.n_runs, c.npop_ctx);
    PA_CHECK_LAUNCH();
    k_parent<<<c.n_chunk_items, CH_THREADS, 0, c.stream>>>(c.chunk_items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    if (c.repr == PA_MSC64) k_copy<PA_MSC64><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs, c.st);
    else k_copy<PA_INT8><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs, c.st);
    return hipGetLastError();
}

int int8_tile_rows(int L)
{
    int T = 512 / L;
    if (T < 1) T = 1;
    if (T > L) T = L;
    return T;
}

size_t msc_lds_bytes(int N) { return (size_t)N * 8 + (size_t)N; }

hipError_t prepare_msc_lds(size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_sweep_msc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_sweep_int8_run(const LaunchCtx &c, int run, int L, int groups_cap, int npop,
                                 int theta)
{
    const int T = int8_tile_rows(L);
    const int ntiles = (L + T - 1) / T;
    const size_t lds = (size_t)(T + 2) * (L / 2) * 8;
    for (int s = 0; s < theta; ++s)
        for (int colour = 0; colour < 2; ++colour)
            for (int p = 0; p < npop; ++p) {
                k_sweep_int8<<<groups_cap * ntiles, 256, lds, c.stream>>>(c.runs, c.st, run, p, s, colour, T,
                                                                          ntiles, c.stats);
                PA_CHECK_LAUNCH();
            }
    return hipSuccess;
}

hipError_t launch_sweep_msc(const LaunchCtx &c, int maxN)
{
    k_sweep_msc<<<c.n_items, 256, msc_lds_bytes(maxN), c.stream>>>(c.items, c.runs, c.st, c.stats);
    return hipGetLastError();
}

hipError_t launch_measure(const LaunchCtx &c)
{
    if (c.repr == PA_MSC64) k_measure<PA_MSC64><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs, c.st);
    else k_measure<PA_INT8><<<c.n_items, 256, 0, c.stream>>>(c.items, c.runs, c.st);
    PA_CHECK_LAUNCH();
    k_finalize<<<c.n_runs, 256, 0, c.stream>>>(c.runs, c.st, c.n_runs, c.npop_ctx);
    return hipGetLastError();
}

hipError_t launch_wavg(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K,
                       int i_done, double *logw, pa_wavg *out)
{
    k_logw<<<(c.n_runs + 255) / 256, 256, 0, c.stream>>>(c.runs, obs, c.n_runs, c.npop_ctx, pop, kind, i_done,
                                                        logw);
    PA_CHECK_LAUNCH();
    const int ng = c.n_runs / M;
    k_wavg<<<(ng * K + 127) / 128, 128, 0, c.stream>>>(c.runs, obs, logw, c.n_runs, c.npop_ctx, pop, M, K, out);
    PA_CHECK_LAUNCH();
    k_wavg_cumsum<<<(ng + 127) / 128, 128, 0, c.stream>>>(out, ng, K);
    return hipGetLastError();
}

}  // namespace pa
