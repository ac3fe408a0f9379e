/*
 * pa.h -- C ABI of the MI355X population-annealing library (libpa.so).
 *
 * Population annealing (PA) with weighted averaging, after Ebert, Gessert and
 * Weigel, "Weighted averages in population annealing: analysis and general
 * framework" (arXiv:2207.05535).  The calls follow the paper's statement of
 * the algorithm, Sec. II B steps (i)-(vi), and of weighted averaging, Sec. IV.
 *
 * Conventions for every call:
 *  - Plain C types only: host pointers are marked "host", device pointers
 *    "device".  No call throws; each returns a pa_status.
 *  - The caller owns the device workspace (one allocation of at least
 *    pa_workspace_size() bytes, 256-byte aligned) and the HIP stream; the
 *    context borrows both until pa_destroy and never allocates device memory
 *    itself.  Host arrays passed in (run descriptors, schedules) are copied.
 *  - Work is enqueued asynchronously on the stream.  Calls that fill host
 *    buffers synchronise the stream before returning.
 *  - Argument validation happens before any device call, so a call rejected
 *    with PA_ERR_ARG or PA_ERR_STATE has enqueued nothing.
 *  - A device failure makes the context sticky-failed (PA_ERR_DEVICE from
 *    then on).  A run whose population overflows its capacity
 *    (PA_ERR_CAPACITY) or becomes empty (PA_ERR_NUMERIC) is frozen: its
 *    later records carry that status, other runs continue, and weighted
 *    averages leave it out.
 *  - Determinism: every result depends only on the run descriptors; not on
 *    batch composition, spin representation, tile shapes or the stream.
 *    Spins, energies, family labels, resampling counts and integer sums are
 *    bit-identical to the plain definitions; ln Q, A and weighted averages
 *    are FP64.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pa_ctx pa_ctx;      /* opaque: one context = a batch of runs */

typedef enum {
    PA_OK = 0,
    PA_ERR_ARG = 1,        /* invalid argument (nothing enqueued) */
    PA_ERR_NOMEM = 2,      /* workspace smaller than pa_workspace_size() */
    PA_ERR_CAPACITY = 3,   /* per run: nearest-integer population exceeded R_cap */
    PA_ERR_STATE = 4,      /* call out of order (nothing enqueued) */
    PA_ERR_NUMERIC = 5,    /* per run: empty population / non-finite input */
    PA_ERR_DEVICE = 6      /* HIP error; the context is unusable */
} pa_status;

/* Models of Sec. III A: Ising ferromagnet (J = 1), Eq. (H_FM), and the
 * Edwards-Anderson +-J spin glass, Eq. (H_EA), on the periodic L x L lattice. */
enum { PA_FM = 0, PA_EA_PMJ = 1 };
/* Resampling of step (iii): multinomial (constant population, Sec. IV D
 * condition (c)) or nearest-integer (Sec. II B). */
enum { PA_MULTINOMIAL = 0, PA_NEAREST_INT = 1 };
/* Spin representation: one byte per spin, or 64 replicas bit-packed per
 * 64-bit word (multi-spin coding).  Results are identical. */
typedef enum { PA_INT8 = 0, PA_MSC64 = 1 } pa_repr;
/* Spin-overlap pairing (Sec. III D): none; index shift j <-> j + floor(R_i/2);
 * two independent populations on the same couplings, pairs j <-> j; or the
 * permutation pairing of Wang et al.: the R_i pairs (k, pi_k) of a random
 * permutation pi repaired so that no pair lies inside one family
 * (PA_Q_WANG), or repaired along a random search pattern (PA_Q_WANG_RDM).
 * The permutations are the index orders of 64-bit Philox keys (counter
 * (k, 0, i, 6 << 28): words 0-1 for pi, 2-3 for the search pattern).  A
 * population with a family of more than R_i / 2 replicas has no such
 * permutation; its record then has no pairs (nPairs = 0). */
enum { PA_Q_NONE = 0, PA_Q_INDEX_SHIFT = 1, PA_Q_TWO_POP = 2, PA_Q_WANG = 3, PA_Q_WANG_RDM = 4 };
/* Free-energy weights, Eq. (appropriateWeight) (full) and Eq. (simpleWeight). */
typedef enum { PA_W_FULL = 0, PA_W_SIMPLE = 1 } pa_weight_kind;
/* Flag OR-ed into a pa_weight_kind argument: overlap averages (W[|q|],
 * W[q^2], W[q_l] and the weighted P(q)) leave out, at each temperature, runs
 * in which a family holds more than R_i / 2 replicas (in either population
 * for PA_Q_TWO_POP), as in the comparison of Sec. III D (Table I); their
 * weights are renormalised over the remaining runs.  The other averages and
 * -beta W[F] are unchanged. */
enum { PA_W_EXCLUDE_LARGE_FAMILY = 2 };

/* One PA run.  Random numbers are drawn from Philox4x32-10 keyed by `seed`
 * (initial spins, sweeps, resampling) and `disorder_seed` (couplings). */
typedef struct {
    int32_t L;              /* linear size: even, 4 <= L <= 1024 (<= 128 for PA_MSC64) */
    int32_t model;          /* PA_FM or PA_EA_PMJ */
    uint64_t seed;          /* run seed */
    uint64_t disorder_seed; /* couplings of PA_EA_PMJ; ignored for PA_FM */
    int32_t R;              /* target population size, >= 1 */
    int32_t R_cap;          /* capacity, R <= R_cap < 2^23; == R for multinomial */
    int32_t theta;          /* Metropolis sweeps per temperature, 0 <= theta < 2^24, or
                               PA_THETA_EXACT (see below) */
    int32_t K;              /* number of temperatures, K >= 2 */
    const double *beta;     /* host [K]: schedule, beta[0] == 0, finite, non-decreasing; copied */
    int32_t resampling;     /* PA_MULTINOMIAL or PA_NEAREST_INT */
    int32_t overlap;        /* PA_Q_NONE, PA_Q_INDEX_SHIFT, PA_Q_TWO_POP, PA_Q_WANG or PA_Q_WANG_RDM */
    int32_t qhist;          /* 1: keep an overlap histogram per temperature */
} pa_run_desc;

/* theta = PA_THETA_EXACT is the theta = infinity limit of Sec. V C: step
 * (iv) replaces every replica's energy by an independent draw from the
 * exact energy distribution g(E) exp(-beta_i E) / Z of the periodic
 * ferromagnet (model PA_FM, L <= 30, overlap PA_Q_NONE).  g comes from
 * pa_exact_dos_wide, each g_m rounded to the nearest double (ties to
 * even); the draw of replica j is v = o0 | o1 << 32 of
 * Philox(seed; j, 0, i, 7 << 28 | pop << 24), and the level is the smallest
 * m with v < C_m, C_m = floor(2^64 S_m / S_N) (2^64 - 1 where S_m = S_N),
 * S_m = sum_{k <= m} (double)g_k exp(-4 beta_i k) in FP64 in increasing k;
 * m = N if there is none.  Only energies are followed: the records' |M|
 * and M^2 sums are zero and the configurations are not updated. */
enum { PA_THETA_EXACT = -1 };

/* Calibration of the integer-VALU ceiling (diagnostic; no context, no
 * device memory): every lane of a grid that fills the device (2048
 * workgroups of 256) runs two independent chains of calls_per_chain
 * Philox4x32-10 calls in registers on hip_stream (NULL: the default
 * stream); *calls_per_s receives the achieved rate, timed with HIP events.
 * A call is 40 VALU instructions (10 rounds of two 32x32->64 multiplies
 * and two three-input XORs), so 40 x *calls_per_s is the lane-op rate the
 * sweep's Philox work can reach.  1 <= calls_per_chain <= 2^20. */
pa_status pa_calibrate_philox(void *hip_stream, int32_t calls_per_chain, double *calls_per_s);

/* Exact density of states of the periodic L x L ferromagnet, the exact
 * energy distribution of the theta = infinity limit (Sec. V C; the paper
 * takes Beale's exact distribution): g_m, the number of configurations with
 * E = -2N + 4m, m = 0..N (N = L^2), from Kaufman's closed form for the
 * torus written as an integer polynomial in exp(-2 beta), evaluated exactly
 * modulo primes and rebuilt by the Chinese remainder theorem (host
 * computation, no device; cached per L).  host_out: [N + 1][limbs]
 * little-endian 64-bit limbs of each g_m; limbs >= N/64 + 1.  L even,
 * 4 <= L <= 30, else PA_ERR_ARG; PA_ERR_NUMERIC if the counts fail their
 * checks (sum 2^N, no odd number of unsatisfied bonds). */
pa_status pa_exact_dos_wide(int32_t L, int32_t limbs, uint64_t *host_out);

/* The same for 4 <= L <= 10 in two limbs: host_out[2m], host_out[2m + 1]
 * receive the low and high 64 bits of g_m. */
pa_status pa_exact_dos(int32_t L, uint64_t *host_out);

/* One record per (run, population, temperature i): integer sums over the
 * population at beta_i (Eqs. (PopAvrg), (e), (m), (c), (chi)), overlaps
 * Q = N q and link overlaps Q_l = 2N q_l per pair, family statistics, and
 * ln Q_i and A_i = -beta_i F_i = sum_{k<=i} ln Q_k + N ln 2 (Eq. (F)). */
typedef struct {
    int64_t R_i;
    double lnQ, A;
    int64_t sumE, sumE2, sumAbsM, sumM2;
    int64_t nPairs, sumQ, sumAbsQ, sumQ2;
    int64_t sumQl, sumQl2;
    int64_t famSumSq, famMax, nFam;   /* rho_t = famSumSq / R_i, Eq. (rho_t) */
    int32_t Emin, status;
} pa_obs;

/* One record per (group of M runs, temperature i), Sec. IV: configurational
 * weighted averages W[e], W[e^2], W[m], W[m^2], W[|q|], W[q^2], W[q_l]
 * (Eq. (W_conf)); weighted variance estimators W_var[c], W_var[chi]
 * (Eqs. (Wvar_C), (Wvar_Chi)) and the configurational averages of c, chi;
 * -beta_i W[F_i] (Eq. (W_F)); the sample variance of the weights and its
 * log-normal prediction (Eq. (varWpred)). */
typedef struct {
    double W_e, W_e2, Wvar_c, Wconf_c, W_m, W_m2, Wvar_chi, Wconf_chi;
    double W_absq, W_q2, W_ql, minus_beta_WF, var_w, var_w_pred;
    int32_t n_included;     /* runs with status PA_OK at this temperature */
} pa_wavg;

/* Family statistics of one (run, population, temperature i), from its
 * record: the mean square family size rho_t = R_i sum_k n_k^2 with n_k the
 * fraction of replicas in family k (Eq. (rho_t)), i.e. sum_k c_k^2 / R_i;
 * the largest family; whether it exceeds R_i / 2; and whether the run is
 * left out of overlap averages at this temperature under
 * PA_W_EXCLUDE_LARGE_FAMILY (a large family in either population of a
 * two-population run, or a status other than PA_OK). */
typedef struct {
    double rho_t;
    int32_t R_i, famMax, large, excluded;
} pa_famstat;

/* Bytes of device workspace needed by pa_create for these runs.
 * runs: host [n_runs]; bytes: host out.  PA_ERR_ARG on an invalid descriptor. */
pa_status pa_workspace_size(const pa_run_desc *runs, int32_t n_runs, pa_repr repr,
                            size_t *bytes);

/* Step (i): draw R configurations from the uniform distribution at beta_0 = 0
 * (Sec. II A), set up couplings, family labels f_j = j and A_0 = N ln 2, and
 * measure at i = 0.  dev_workspace: device, >= pa_workspace_size bytes, owned
 * by the caller; hip_stream: a hipStream_t (NULL = default stream).
 * On success *out receives the context. */
pa_status pa_create(const pa_run_desc *runs, int32_t n_runs, pa_repr repr,
                    void *dev_workspace, size_t bytes, void *hip_stream, pa_ctx **out);

/* Size of the library's own device workspace used by pa_create_static. */
#define PA_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)

/* pa_create without a caller-provided workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The context lives in a device array of
 * PA_STATIC_WORKSPACE_BYTES that the library holds on each GPU it runs on
 * until the process ends; this call allocates no device memory.  Runs needing
 * more than that (pa_workspace_size) are rejected with PA_ERR_NOMEM before
 * any device call.  The array is shared by every caller on one GPU: while a
 * context created here is alive, a second pa_create_static on the same
 * device returns PA_ERR_STATE; pa_destroy releases it.  The workspace is
 * cleared at creation, so nothing from an earlier context carries over.
 * Work of two contexts on one GPU's array must not overlap in time (it would
 * race); the PA_ERR_STATE check enforces this for contexts of this process.
 * Every other entry point works on the returned context as on one from
 * pa_create; results are identical. */
pa_status pa_create_static(const pa_run_desc *runs, int32_t n_runs, pa_repr repr, void *hip_stream,
                           pa_ctx **out);

/* Step (ii) for i = previous + 1: Q_i of Eq. (QBoltz) from the energies at
 * beta_{i-1}, ln Q_i and A_i (Eq. (F)), and the resampling weights of
 * Eq. (tauBoltz).  Requires the previous step to have been measured. */
pa_status pa_anneal_step(pa_ctx *ctx, int32_t i);

/* Step (iii): descendant counts (nearest-integer or multinomial), their
 * prefix scan, and the copy of spins, energies and family labels into
 * consecutive child slots, so that families stay contiguous (Sec. V A 1). */
pa_status pa_resample(pa_ctx *ctx, int32_t i);

/* Step (iv): theta checkerboard single-spin-flip Metropolis sweeps at beta_i
 * (Sec. V A 1).  PA_INT8 contexts launch one colour of one run at a time;
 * PA_MSC64 contexts update every run in one launch with the lattice held in
 * on-chip memory for all theta sweeps. */
pa_status pa_sweep(pa_ctx *ctx, int32_t i);

/* Step (v): energies, magnetisations, overlaps and family sizes at beta_i.
 * host_out: host [n_runs][n_pop] records of temperature i, or NULL
 * (n_pop = 2 for every run when any run uses PA_Q_TWO_POP, else 1; the
 * second slot of a one-population run is zero). */
pa_status pa_measure(pa_ctx *ctx, int32_t i, pa_obs *host_out);

/* Steps (ii)-(v) for i = i_begin .. i_end-1, replayed from one captured HIP
 * graph of a temperature step.  Requires i_begin = previous + 1. */
pa_status pa_run(pa_ctx *ctx, int32_t i_begin, int32_t i_end);

/* Sec. IV: weighted averages over consecutive groups of M runs (runs
 * [gM, (g+1)M) form group g; n_runs % M == 0; every run of a group must have
 * the same L and schedule).  pop selects the population whose records are
 * weighted.  host_out: host [n_runs/M][K].  Computed in FP64 on the device
 * from the records of temperatures 0..i of the steps done so far; records of
 * temperatures not reached yet are reported with n_included = 0.  kind:
 * PA_W_FULL or PA_W_SIMPLE, optionally | PA_W_EXCLUDE_LARGE_FAMILY. */
pa_status pa_weighted_average(pa_ctx *ctx, int32_t M, int32_t kind, int32_t pop,
                              pa_wavg *host_out);

/* Sec. IV C, Eq. (W_conf_q): the weighted overlap distribution
 * W[P(q)] = sum_m w^(m) P^(m)(q) of each group of M consecutive runs (every
 * run of a group needs qhist = 1, the same L and schedule), with P^(m) the
 * empirical distribution of run m's overlap pairs (its histogram divided by
 * its number of pairs) and the free-energy weights of `kind` (PA_W_FULL or
 * PA_W_SIMPLE, optionally | PA_W_EXCLUDE_LARGE_FAMILY).  Bin d is Hamming
 * distance d, q = 1 - 2d/N.  host_out: host [n_runs/M][K][N+1]; temperatures
 * not reached yet, or with no included run, are NaN.  FP64 on the device. */
pa_status pa_weighted_qhist(pa_ctx *ctx, int32_t M, int32_t kind, int32_t pop, double *host_out);

/* Family statistics of every run of population pop at every temperature
 * reached (pa_famstat above).  host_out: host [n_runs][K]. */
pa_status pa_family_stats(pa_ctx *ctx, int32_t pop, pa_famstat *host_out);

/* All records so far.  host_out: host [n_runs][n_pop][K]. */
pa_status pa_read_obs(pa_ctx *ctx, pa_obs *host_out);

/* Overlap histograms of one run (qhist = 1): host [n_pop][K][N+1] int32,
 * bin d = number of pairs at Hamming distance d (q = 1 - 2d/N). */
pa_status pa_read_qhist(pa_ctx *ctx, int32_t run, int32_t *host_out);

/* Permutation pairing of a PA_Q_WANG / PA_Q_WANG_RDM run at the last
 * measured temperature (Sec. III D): host_pairs host [R_cap] int32 receives
 * the partner pi_k of every replica k < R_i; *status (may be NULL) receives
 * 0, or 1 when a family held more than R_i / 2 replicas (no pairing; pairs
 * left unspecified), and *R_i (may be NULL) the population size.  Needs the
 * context in its measured state (PA_ERR_STATE otherwise); PA_ERR_ARG for a
 * run with another overlap kind. */
pa_status pa_read_pairing(pa_ctx *ctx, int32_t run, int32_t *host_pairs, int32_t *status, int32_t *R_i);

/* Current population of (run, pop) in canonical form: spins host
 * [R_cap][N] int8 (+1/-1, replica-major, site n = y L + x), energies and
 * family labels host [R_cap] int32, descendant counts of the last
 * resampling host [R_cap] int32; any pointer may be NULL.  *R_i and *R_prev
 * (may be NULL) receive the current and previous population sizes. */
pa_status pa_read_state(pa_ctx *ctx, int32_t run, int32_t pop, int8_t *spins, int32_t *E,
                        int32_t *fam, int32_t *counts, int32_t *R_i, int32_t *R_prev);

/* Checkpoint: with host_buf == NULL, *bytes receives the size needed; else
 * the complete run state is written to host_buf (size *bytes). */
pa_status pa_checkpoint(pa_ctx *ctx, void *host_buf, size_t *bytes);

/* Restore a checkpoint taken from a context created with the same
 * descriptors and representation.  Continuing from it reproduces the
 * uninterrupted run bit for bit.  The checkpoint carries a hash of every run
 * descriptor and schedule: a checkpoint of other runs (another seed, theta,
 * model, schedule, ...) is rejected with PA_ERR_ARG and the context is left
 * unchanged.  The launch shapes are the context's own, not the checkpoint's:
 * a restore after pa_set_tuning, pa_set_persistent or pa_set_sweep_chunks
 * (or into another context with other shapes) continues with the current
 * ones, and the results do not depend on them. */
pa_status pa_restore(pa_ctx *ctx, const void *host_buf, size_t bytes);

/* Launch-shape knobs of the batched sweep, chosen by the autotuner per
 * lattice size L: threads per workgroup (64..1024, a power of two, shared by
 * all L of the context), replica groups per workgroup for this L, and the
 * number of Philox calls every site makes in lockstep before the undecided
 * sites are compacted (0..16).  A shape that does not fit the device is
 * rejected with PA_ERR_ARG and the previous shape is kept.  Results never
 * depend on the shape. */
pa_status pa_set_tuning(pa_ctx *ctx, int32_t L, int32_t threads, int32_t groups_per_wg,
                        int32_t dense_calls);

/* Persistent grid for the batched sweep: on = 1 launches as many
 * workgroups as the device holds at once, each taking items (largest lattice
 * block first) from a device ticket counter until none is left; on = 0
 * launches one workgroup per item (the hardware dispatcher hands them out in
 * the same largest-first order).  Results never depend on it. */
pa_status pa_set_persistent(pa_ctx *ctx, int32_t on);

/* Sweep chunks on the persistent grid: chunks = K > 1 splits every item of
 * the batched sweep into K items of consecutive sweeps (chunk c takes sweeps
 * c theta / K .. (c + 1) theta / K - 1 of its replica groups), listed all
 * first chunks first; a chunk waits on the device until the previous chunk
 * of its groups has stored their lattices.  With every item taking about the
 * same time, a launch of n items on S resident workgroups lasts about
 * ceil(n / S) item times; chunks bring that down to ceil(n K / S) / K at the
 * cost of loading and storing each lattice K - 1 more times, which for
 * small items can outweigh the gain.  1 <= chunks <= 4 fixes K (default 1;
 * pa_autotune searches it); chunks = 0 chooses K per plan from the estimate
 * above.  Chunks apply only where the persistent grid is used
 * (pa_set_persistent, and more items than resident workgroups).  Results
 * never depend on it.  PA_ERR_ARG outside 0..4, PA_ERR_STATE between the
 * calls of a temperature step. */
pa_status pa_set_sweep_chunks(pa_ctx *ctx, int32_t chunks);

/* Chunks per item of the current sweep plan (host *out: 1 when items are
 * whole). */
pa_status pa_get_sweep_chunks(pa_ctx *ctx, int32_t *out);

/* Launches of the batched sweep per temperature step in the current plan
 * (host *out): 0 without Metropolis sweeps; 1 when the sweeping runs share
 * one lattice size and model, or for a mix that one dispatching kernel
 * serves; one per (size, model) when the runs mix sizes that each have a
 * kernel of their own and every size fills at least half of the
 * workgroups its kernel keeps resident.  Results never depend on it. */
pa_status pa_get_sweep_launches(pa_ctx *ctx, int32_t *out);

/* Sparse rounds of the batched sweep: on = 1 pools the sites still
 * undecided after the lockstep calls into one list per workgroup, so the
 * compacted rounds run on full wavefronts; on = 0 keeps one list per
 * wavefront (no workgroup barriers in those rounds).  Results never depend
 * on it. */
pa_status pa_set_pooled(pa_ctx *ctx, int32_t on);

/* Current launch shape of the batched sweep for lattice size L (any output
 * pointer may be NULL). */
pa_status pa_get_tuning(pa_ctx *ctx, int32_t L, int32_t *threads, int32_t *groups_per_wg,
                        int32_t *dense_calls, int32_t *persistent, int32_t *pooled);

/* Autotuner of the batched sweep (no-op for the plain path).  From the
 * current state (all steps so far measured) it runs `steps` (1..64, clipped
 * to the remaining schedule) real temperature steps of this context for
 * each candidate launch shape, timing the sweep launches with HIP events:
 * first threads x dense_calls x persistent x pooled with the current groups per L,
 * then groups per workgroup one L at a time (heaviest L first), then, with a
 * persistent grid, 2..4 chunks of sweeps per item.  Every
 * candidate's records and exact work counters must hash to the starting
 * shape's value; one that differs is rejected (counted in *n_rejected, which
 * is 0 unless a kernel is wrong).  The fastest accepted shape is applied and
 * the context is returned to its starting state, so the tuned run continues
 * exactly as an untuned one would.  Takes a pinned host snapshot of the
 * workspace for the duration of the call.
 * cache_path (host string, may be NULL): JSON file of shapes keyed by
 * (device architecture, representation, L).  If it holds every L of the
 * context, those shapes are applied without a search (*n_tried = 0); after a
 * search the chosen shape is merged into it.  A cache that cannot be written
 * gives PA_ERR_ARG after the shape has been applied. */
pa_status pa_autotune(pa_ctx *ctx, int32_t steps, const char *cache_path, int32_t *n_tried,
                      int32_t *n_rejected);

/* Exact work counters of the sweep kernels since pa_create: host_out[3] =
 * {site updates of 64-replica words, Philox4x32-10 calls, attempted
 * single-spin flips}.  Used to express sweep throughput against the
 * integer-ALU roofline.  Returns PA_ERR_STATE (counters still written) if a
 * sweep chunk ever gave up waiting for the chunk before it (see
 * pa_set_sweep_chunks) or a sweep item was skipped for not fitting the
 * launch's LDS (a device work list out of step with the plan; never expected):
 * the steps since then are not to be trusted. */
pa_status pa_read_stats(pa_ctx *ctx, uint64_t *host_out);

/* ------------------------------------------------------------------ serving
 *
 * Continuous batching of independent runs (a stream of requests, each one
 * PA run of Sec. II B).  A server owns a caller-allocated device arena
 * (256-byte aligned; borrowed until pa_server_destroy) and max_slots slots.
 * Runs are admitted while a slot is free and their footprint fits in the
 * free arena space; each server step advances every resident run that has
 * not reached its last temperature by one temperature step (steps ii-v),
 * whatever temperature it is at, in shared launches.  A run's records equal
 * those of the same descriptor run alone in a pa_ctx, bit for bit.  All work
 * goes to the caller's stream in order; a server is used from one host
 * thread at a time. */
typedef struct pa_server pa_server;

/* Device bytes one run takes in a server arena: its own block (populations,
 * records, work lists) plus its tables, which it shares with resident runs
 * of the same L and schedule (so the bound is not always reached).
 * PA_ERR_ARG for an invalid descriptor. */
pa_status pa_server_footprint(const pa_run_desc *desc, pa_repr repr, size_t *bytes);

/* tuning_cache (host string, may be NULL): autotuner cache file whose shapes
 * the batched sweep uses (see pa_autotune).  PA_ERR_NOMEM if the arena
 * cannot hold the slot table. */
pa_status pa_server_create(pa_repr repr, void *dev_arena, size_t arena_bytes, int32_t max_slots,
                           const char *tuning_cache, void *hip_stream, pa_server **out);

/* Admits one run and enqueues its step (i) and the measurement at i = 0.
 * *slot receives its slot.  PA_ERR_CAPACITY: no free slot; PA_ERR_NOMEM:
 * its footprint does not fit in the free arena space now (nothing changed;
 * retry after a release). */
pa_status pa_server_admit(pa_server *srv, const pa_run_desc *desc, int32_t *slot);

/* Enqueues one temperature step for every resident run that has not
 * reached its last temperature.  finished (host, capacity max_slots)
 * receives the slots whose run reached its last temperature in this step
 * (*n_finished of them); their records are complete once the stream has
 * passed this step. */
pa_status pa_server_step(pa_server *srv, int32_t *finished, int32_t *n_finished);

/* Temperature index a resident run has been advanced to (as enqueued). */
pa_status pa_server_progress(pa_server *srv, int32_t slot, int32_t *i_done);

/* Copies a resident run's records to host_out (host [K][n_pop]).  sync = 1
 * waits for the copy; sync = 0 only enqueues it (host_out should then be
 * pinned memory and must not be read before the stream has passed it). */
pa_status pa_server_read_obs(pa_server *srv, int32_t slot, pa_obs *host_out, int32_t sync);

/* Frees a slot and its arena space for later admissions.  Work already
 * enqueued for it (including an unsynchronised pa_server_read_obs) still
 * completes first. */
pa_status pa_server_release(pa_server *srv, int32_t slot);

/* Occupancy: resident runs, arena bytes in use, largest free extent (any
 * pointer may be NULL). */
pa_status pa_server_info(pa_server *srv, int32_t *resident, size_t *bytes_used, size_t *largest_free);

const char *pa_server_last_error(pa_server *srv);

/* Synchronises the stream and releases the server (not the arena). */
pa_status pa_server_destroy(pa_server *srv);

/* Text of the first HIP error that made the context fail ("none" if it has
 * not failed).  The string is static; do not free it. */
const char *pa_last_error(pa_ctx *ctx);

/* Releases the context (not the workspace or the stream). */
pa_status pa_destroy(pa_ctx *ctx);

const char *pa_status_str(pa_status st);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
