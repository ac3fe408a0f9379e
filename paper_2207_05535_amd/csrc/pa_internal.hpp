// pa_internal.hpp -- device-side data model shared by the host code and the
// kernels of libpa.so.
//
// Everything a kernel needs about a run lives in a RunInfo record in device
// memory (constant after creation), and everything that changes from step to
// step lives in a PopState record per (run, population).  Kernels read the
// temperature index, the current spin buffer and the population size from
// PopState, so a temperature step is a fixed sequence of launches whose
// arguments never change: it can be captured once as a HIP graph and
// replayed for every step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pa.h"

namespace pa {

// Philox counter tags: the top nibble of the fourth counter word says what a
// draw is for, so draws for different purposes never collide.
constexpr uint32_t TAG_SWEEP = 1u;
constexpr uint32_t TAG_NI = 2u;
constexpr uint32_t TAG_MN = 3u;
constexpr uint32_t TAG_INIT = 4u;
constexpr uint32_t TAG_J = 5u;
constexpr uint32_t TAG_PERM = 6u;
constexpr uint32_t TAG_DOS = 7u;

constexpr int MAX_POP = 2;

// Population-wide scans and reductions work on chunks of CH replicas: one
// workgroup of CH_THREADS threads, CH_PER consecutive replicas per thread.
constexpr int CH_THREADS = 256;
constexpr int CH_PER = 8;
constexpr int CH = CH_THREADS * CH_PER;
constexpr int NACC = 13;  // measure accumulators, see Acc

// Measurement: workgroups of MEAS_WAVES wavefronts; a lattice of N sites
// gets one wavefront per group up to 1024 sites, two up to 2048, else four.
constexpr int MEAS_WAVES = 4;
constexpr int MEAS_THREADS = 64 * MEAS_WAVES;
// The measurement stages a workgroup's lattices in LDS up to this many sites
// per lattice: MEAS_WAVES / waves-per-group lattices of N words, at most
// 4096 x 8 bytes (one group of 4096 sites, or four of 1024).
constexpr int MEAS_STAGE_N = 4096;
constexpr size_t MEAS_STAGE_BYTES = 32768;
// per-group partial sums: E, E^2, |M|, M^2, pairs, Q, |Q|, Q^2, Q_l, Q_l^2,
// minimum energy
constexpr int MEAS_PART = 11;

__host__ __device__ inline int meas_waves_per_group(int N) { return N <= 1024 ? 1 : (N <= 2048 ? 2 : 4); }

enum Acc { A_SUME = 0, A_SUME2, A_SUMABSM, A_SUMM2, A_NPAIRS, A_SUMQ, A_SUMABSQ, A_SUMQ2,
           A_SUMQL, A_SUMQL2, A_FAMSQ, A_FAMMAX, A_NFAM };

struct RunInfo {
    int32_t L, N, npop, R, R_cap, theta, K, model, resampling, overlap, qhist, groups_cap;
    uint32_t key0, key1;
    // record of (population p, temperature i): obs[i * obs_stride + obs_off + p]
    int32_t obs_stride, obs_off;
    int32_t wang_lb;              // permutation pairing: log2 of the bucket capacity
    int32_t exact_dos;            // 1: theta = infinity (energies drawn; theta is 0 here)
    // device pointers into the caller's workspace
    uint8_t *spins[MAX_POP][2];   // int8: [group][site][64] bytes; MSC: [group][site] u64
    int32_t *E[MAX_POP][2];       // energies [R_cap]
    int32_t *fam[MAX_POP][2];     // family labels [R_cap]
    int32_t *r[MAX_POP];          // descendant counts [R_cap]
    int32_t *C[MAX_POP];          // exclusive prefix of r [R_cap + 1]
    int32_t *parent[MAX_POP];     // child -> parent [R_cap]
    uint64_t *P[MAX_POP];         // multinomial prefix of X [R_cap + 1]
    int64_t *part[MAX_POP];       // per group: MEAS_PART partial sums of the measurement
    double *partS[MAX_POP];       // per chunk: partial sum of x_j
    uint64_t *tot64[MAX_POP];     // per chunk: sum of X_j
    uint64_t *base64[MAX_POP];    // per chunk: exclusive prefix of tot64
    int32_t *tot32[MAX_POP];      // per chunk: sum of r_j
    int32_t *base32[MAX_POP];     // per chunk: exclusive prefix of tot32
    pa_obs *obs;                  // records, indexed through obs_stride and obs_off
    int32_t *qh;                  // [n_pop][K][N+1] or nullptr
    uint8_t *jbits;               // [N]: bit0 = J_R(n) < 0, bit1 = J_D(n) < 0
    int32_t *wang;                // permutation pairing scratch (see WangBufs) or nullptr
    const uint64_t *tabD;         // theta = infinity: energy draw thresholds [K][N+1] or nullptr
    const uint64_t *tabX;         // [K][N+1]  floor(exp(-dbeta_i 4k) 2^40)
    const double *tabx;           // [K][N+1]  exp(-dbeta_i 4k)
    const uint64_t *tabT;         // [K][2]    Metropolis thresholds for dE = 4, 8
    const double *beta;           // [K]
};

struct PopState {
    int32_t i;        // temperature index of the current population
    int32_t cur;      // current spin buffer (0/1)
    int32_t src;      // buffer the last resampling copied from
    int32_t Rprev;    // population size before the last resampling
    int32_t Rcur;     // current population size
    int32_t status;   // PA_OK or a sticky per-run failure
    int32_t Emin;     // minimum energy of the current population
    int32_t moved;    // 1 if this population advanced in the current step
    double lnQ, A, S;
    uint64_t SX;
    int64_t acc[NACC];
    int32_t EminAcc;
    int32_t pad1;
};

// Work counters of the sweep kernels (exact, for the ALU roofline):
// word-site updates (64 replicas of one site), Philox calls, attempted flips.
// They are striped over STAT_SLOTS slots of 64 bytes (NSTAT counters each)
// so that concurrent wavefronts add to different cache lines; a reader sums
// the slots.
enum Stat { ST_WORDS = 0, ST_CALLS = 1, ST_FLIPS = 2, ST_STALL = 3, NSTAT = 8 };
constexpr int STAT_SLOTS = 256;
constexpr size_t STAT_BYTES = sizeof(uint64_t) * NSTAT * STAT_SLOTS;

struct Item {         // one replica group (64 replicas) of one (run, pop)
    int32_t run, pop, group, pad;
};

struct SweepItem {    // groups [group0, group0 + ngroups) of one (run, pop), one workgroup
    int32_t run, pop, group0, ngroups;
    // chunk `chunk` of `nchunk` of those groups' theta sweeps (nchunk <= 1:
    // all of them): with two chunks, sweeps 0 .. cut - 1 and cut .. theta - 1;
    // with more, as even as possible, the larger first.  chunk > 0 waits for
    // the previous chunk of the same groups, whose completion is published in
    // flag slot `base`
    int32_t chunk, nchunk, base, cut;
};
constexpr int MAX_SWEEP_CHUNKS = 4;

// LDS bytes of a batched-sweep workgroup holding `groups` replica groups of
// N sites: the colour-split lattices, the lists of undecided sites (two
// 64-bit masks and a 32-bit entry per unit), the bond signs and the counters.
// Queue slots per wavefront of the streamed sparse rounds: a wavefront
// that owns more site words than this keeps its undecided sites in a ring
// of this many entries, run down by full rounds whenever it holds more than
// one chunk's worth (a chunk adds at most 64, and full rounds leave at most
// 64), so the lists take less LDS and more workgroups fit on a CU.
constexpr int MSC_QUEUE_SLOTS = 128;
constexpr int MSC_WHOLE_LISTS = 1 << 9;

// mode = lockstep calls | pooled << 8 | whole lists << 9, as the batched
// sweep is launched (whole lists: one entry per site word even when the
// rounds are streamed; the kernel that dispatches per item uses them, its
// many registers leaving no room for more workgroups per CU anyway).  The
// sparse rounds are streamed for lattices of at most 4096 sites when they
// are not pooled and there are sparse rounds at all.
__host__ __device__ inline bool msc_streamed(int N, int mode)
{
    return !((mode >> 8) & 1) && N <= 4096 && (mode & 0xFF) < 16;
}

// Entries of a workgroup's lists of undecided sites: one per site word of
// one colour of its groups, or MSC_QUEUE_SLOTS per wavefront when streamed
// rounds let that be fewer.
__host__ __device__ inline int msc_list_entries(int N, int groups, int nw, int mode)
{
    const int units = groups * (N / 2);
    const int upw = (units + nw - 1) / nw;
    return msc_streamed(N, mode) && !(mode & MSC_WHOLE_LISTS) && upw > MSC_QUEUE_SLOTS ? nw * MSC_QUEUE_SLOTS
                                                                                        : units;
}

// Layout: lattices [groups][N] u64, undecided lanes of the two classes
// [entries] u64 each, list entries [entries] u32, bond signs [N] u8 (spin
// glass only), list counts [34] int, then (16-byte aligned) T's bits at the
// planes of each call [16] uint4.  nw: wavefronts of the workgroup.
__host__ __device__ inline size_t msc_lds_tmask_off(int N, int groups, bool ea, int nw, int mode)
{
    const size_t ent = (size_t)msc_list_entries(N, groups, nw, mode);
    const size_t end = (size_t)groups * N * 8 + ent * 20 + (ea ? (size_t)N : 0) + sizeof(int) * 34;
    return (end + 15) & ~(size_t)15;
}

__host__ __device__ inline size_t msc_lds_need(int N, int groups, bool ea, int nw, int mode)
{
    return msc_lds_tmask_off(N, groups, ea, nw, mode) + 16 * 16;
}

struct ChunkItem {    // one chunk of CH replicas of one (run, pop)
    int32_t run, pop, chunk, pad;
};

__host__ __device__ inline int n_pop_of(int overlap) { return overlap == PA_Q_TWO_POP ? 2 : 1; }
__host__ __device__ inline bool is_wang(int overlap) { return overlap == PA_Q_WANG || overlap == PA_Q_WANG_RDM; }

// Permutation-pairing scratch of a run (int32 units), B = 2^wang_lb >= R_cap:
// pi, sigma, fam[pi], bucket members, mismatch list [R_cap] each; bucket
// counts [B]; bucket starts [B + 1]; header [4] (status: 0 paired, 1 a
// family above R_i / 2, 2 no partner found; mismatch count); then, 8-byte
// aligned, the bit rows of the population (64-bit words).
__host__ __device__ inline int wang_lb_of(int R_cap)
{
    int lb = 1;
    while ((1 << lb) < R_cap) ++lb;
    return lb;
}
__host__ __device__ inline size_t wang_ints_head(int R_cap)   // the int32 arrays, even count
{
    return (5 * (size_t)R_cap + 2 * ((size_t)1 << wang_lb_of(R_cap)) + 1 + 4 + 1) & ~(size_t)1;
}
// Bit rows of the population (see k_wang_rows): ceil(N/64) blocks of
// 64 groups_cap words, after the int32 arrays.
__host__ __device__ inline size_t wang_row_words(int R_cap, int N)
{
    return (size_t)((N + 63) / 64) * (size_t)(((R_cap + 63) / 64) * 64);
}
__host__ __device__ inline size_t wang_ints(int R_cap, int N) { return wang_ints_head(R_cap) + 2 * wang_row_words(R_cap, N); }
__host__ __device__ inline uint64_t *wang_rows(int32_t *w, int R_cap) { return (uint64_t *)(w + wang_ints_head(R_cap)); }
struct WangBufs {
    int32_t *pi, *sigma, *fampi, *members, *list, *cnt, *start, *hdr;
};
__host__ __device__ inline WangBufs wang_bufs(int32_t *w, int R_cap, int lb)
{
    WangBufs b;
    b.pi = w;
    b.sigma = b.pi + R_cap;
    b.fampi = b.sigma + R_cap;
    b.members = b.fampi + R_cap;
    b.list = b.members + R_cap;
    b.cnt = b.list + R_cap;
    b.start = b.cnt + ((size_t)1 << lb);
    b.hdr = b.start + ((size_t)1 << lb) + 1;
    return b;
}

}  // namespace pa
