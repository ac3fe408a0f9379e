/*
 * pa_oracle.c -- CPU oracle for population annealing (PA) with weighted
 * averaging, after Ebert, Gessert and Weigel, "Weighted averages in
 * population annealing: analysis and general framework" (arXiv:2207.05535).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the GPU path.
 *
 * What it computes, step by step (Sec. II B, steps (i)-(vi)):
 *   (i)   R_0 = R configurations drawn uniformly at beta_0 = 0.
 *   (ii)  Q_i, Eq. (QBoltz); the free-energy estimator of Eq. (F):
 *         A_i = -beta_i F_i = sum_k ln Q_k + ln Z(beta_0), ln Z(0) = N ln 2.
 *   (iii) resampling with mean tau_i^(j), Eq. (tauBoltz): nearest-integer
 *         (Sec. II B) or multinomial (Sec. IV C, condition (c)); copies of one
 *         parent placed next to each other (Sec. V A 1).
 *   (iv)  theta checkerboard single-spin-flip Metropolis sweeps (Sec. V A 1).
 *   (v)   population averages, Eqs. (PopAvrg), (e), (m), (c), (chi), and spin
 *         overlaps (Sec. III D): index shift floor(R_i/2), two populations,
 *         or the permutation pairing of Wang et al. (with or without a
 *         random search pattern).
 *   Sec. IV: free-energy weights, Eqs. (appropriateWeight), (simpleWeight);
 *         configurational averages, Eq. (W_conf); weighted variance,
 *         Eqs. (Wvar_C), (Wvar_Chi), (Wvar_bound); weighted free energy,
 *         Eq. (W_F); log-normal weight-variance prediction, Eq. (varWpred).
 *
 * Random numbers.  PA is stochastic, so "the result" of a run is the
 * algorithm executed under a fixed random-number and arithmetic contract.
 * All draws come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * written here from that published definition, keyed by the run seed and
 * addressed by a counter that names what the draw is for.  The contract
 * (counter layout, bit-plane assembly of the Metropolis draw, threshold and
 * reweighting tables, integer resampling arithmetic) is stated at each use.
 *
 * Parity pins: see tests/test_oracle_*.py.  Functions without an external
 * pin say so in their comment ("parity unpinned").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- types -- */

typedef struct {
    int32_t L;              /* linear lattice size, even, N = L*L */
    int32_t model;          /* 0 = ferromagnet, 1 = +-J spin glass */
    uint64_t seed;          /* run seed: Philox key for init/sweep/resample */
    uint64_t disorder_seed; /* Philox key for the couplings (spin glass) */
    int32_t R;              /* target population size */
    int32_t R_cap;          /* capacity (>= R) */
    int32_t theta;          /* sweeps per temperature; -1: theta = infinity, the
                               energies drawn from the exact distribution
                               at beta_i (ferromagnet, L <= 30, no overlaps;
                               for L > 8 the density of states is supplied
                               with or_set_dos) */
    int32_t K;              /* number of temperatures beta[0..K-1] */
    const double *beta;     /* annealing schedule, beta[0] = 0 */
    int32_t resampling;     /* 0 = multinomial, 1 = nearest integer */
    int32_t overlap;        /* 0 none, 1 index shift, 2 two populations,
                               3 permutation pairing, 4 the same with a
                               random search pattern */
    int32_t qhist;          /* 1: keep overlap histograms per temperature */
} or_desc;

typedef struct {            /* one per (population, temperature) */
    int64_t R_i;
    double lnQ, A;          /* A = -beta_i F_i */
    int64_t sumE, sumE2, sumAbsM, sumM2;
    int64_t nPairs, sumQ, sumAbsQ, sumQ2;
    int64_t sumQl, sumQl2;
    int64_t famSumSq, famMax, nFam;
    int32_t Emin, status;
} or_obs;

typedef struct {            /* one per temperature of a group of runs */
    double W_e, W_e2, Wvar_c, Wconf_c, W_m, W_m2, Wvar_chi, Wconf_chi;
    double W_absq, W_q2, W_ql, minus_beta_WF, var_w, var_w_pred;
    int32_t n_included;
} or_wavg;

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_CAPACITY = 3, OR_ERR_STATE = 4,
       OR_ERR_NUMERIC = 5 };

enum { TAG_SWEEP = 1u, TAG_NI = 2u, TAG_MN = 3u, TAG_INIT = 4u, TAG_J = 5u, TAG_PERM = 6u, TAG_DOS = 7u };

enum { PH_MEASURED = 0, PH_ANNEALED = 1, PH_RESAMPLED = 2, PH_SWEPT = 3 };

typedef struct {
    int8_t *s[2];           /* spins, ping-pong, [R_cap][N], values +1/-1 */
    int32_t *E[2];          /* energies, tracked through the sweeps */
    int32_t *f[2];          /* family label = index of the ancestor at beta_0 */
    int cur;
    int32_t Rcur;           /* population size at the current temperature */
    int32_t Rprev;          /* population size before the last resampling */
    int32_t *r;             /* descendants per replica of the last resampling */
    uint64_t *X;            /* integer reweighting factor per replica */
    double A, lnQ;
    uint64_t SX;
    int32_t status;
    int32_t Emin;
} or_pop;

typedef struct {
    or_desc d;
    double *beta;
    int N, npop;
    uint32_t key[2];
    int8_t *jR, *jD;        /* couplings of the bonds (n, right(n)), (n, down(n)) */
    or_pop pop[2];
    or_obs *obs;            /* [npop][K] */
    int32_t *qh;            /* [npop][K][N+1] or NULL */
    double *rho;            /* [npop][K] mean square family size, Eq. (rho_t) */
    uint64_t *dosC;         /* theta = infinity: energy draw thresholds [K][N+1] */
    int i, phase;
    int64_t e_mismatch;     /* tracked-vs-recomputed energy mismatches seen */
} or_run;

/* --------------------------------------------------------------- Philox -- */

/* Philox4x32 with 10 rounds, as published by Salmon et al. (SC'11): each
 * round multiplies the even counter words by two fixed odd constants, takes
 * the 64-bit products apart, mixes the high halves with the odd counter
 * words and the key, and permutes; the key is advanced by two Weyl
 * increments between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void key_of(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

static void philox_at(const uint32_t key[2], uint32_t a, uint32_t b, uint32_t c,
                      uint32_t d, uint32_t out[4])
{
    uint32_t ctr[4] = {a, b, c, d};
    or_philox4x32_10(ctr, key, out);
}

/* --------------------------------------------------------------- tables -- */

/* Metropolis threshold for an energy increase dE > 0 at inverse temperature
 * beta: the move is accepted iff a uniform 32-bit draw u satisfies u < T,
 * with T = floor(exp(-beta dE) * 2^32) in [0, 2^32], computed in double with
 * the C library exp.  T / 2^32 differs from exp(-beta dE) by less than 2^-32. */
uint64_t or_sweep_threshold(double beta, int dE)
{
    double p = exp(-(beta * (double)dE));
    return (uint64_t)floor(ldexp(p, 32));
}

/* Reweighting factor of a replica whose energy is E_min + 4k, for the step
 * beta_{i-1} -> beta_i with dbeta = beta_i - beta_{i-1}, Eq. (tauBoltz):
 * x = exp(-dbeta (E - E_min)) in double, and its integer image
 * X = floor(x 2^40) used for resampling. */
double or_reweight_x(double dbeta, int k)
{
    return exp(-(dbeta * (double)(4 * k)));
}

uint64_t or_reweight_X(double dbeta, int k)
{
    return (uint64_t)floor(ldexp(or_reweight_x(dbeta, k), 40));
}

/* -------------------------------------------------------------- lattice -- */

static int right_of(int n, int L) { int x = n % L, y = n / L; return y * L + (x + 1) % L; }
static int left_of(int n, int L)  { int x = n % L, y = n / L; return y * L + (x + L - 1) % L; }
static int down_of(int n, int L)  { int x = n % L, y = n / L; return ((y + 1) % L) * L + x; }
static int up_of(int n, int L)    { int x = n % L, y = n / L; return ((y + L - 1) % L) * L + x; }

/* Energy of one configuration, Eqs. (H_FM)/(H_EA): each of the 2N bonds
 * (n, right(n)) and (n, down(n)) counted once. */
static int32_t energy_of(const or_run *run, const int8_t *s)
{
    int L = run->d.L, N = run->N;
    int32_t E = 0;
    for (int n = 0; n < N; n++) {
        E -= run->jR[n] * s[n] * s[right_of(n, L)];
        E -= run->jD[n] * s[n] * s[down_of(n, L)];
    }
    return E;
}

static int32_t magnetisation_of(const or_run *run, const int8_t *s)
{
    int32_t M = 0;
    for (int n = 0; n < run->N; n++) M += s[n];
    return M;
}

/* ---------------------------------------------------------------- create -- */

static void obs_frozen(or_obs *o, int32_t status)
{
    memset(o, 0, sizeof(*o));
    o->status = status;
}

static int measure_impl(or_run *run, int i);

void or_destroy(or_run *run)
{
    if (!run) return;
    for (int p = 0; p < 2; p++) {
        for (int b = 0; b < 2; b++) {
            free(run->pop[p].s[b]);
            free(run->pop[p].E[b]);
            free(run->pop[p].f[b]);
        }
        free(run->pop[p].r);
        free(run->pop[p].X);
    }
    free(run->jR); free(run->jD);
    free(run->beta); free(run->obs); free(run->qh); free(run->rho); free(run->dosC);
    free(run);
}

/* ------------------------------------------ theta = infinity limit -- */

/* Exact density of states of the periodic L x L ferromagnet, the input of
 * the theta = infinity limit (Sec. V C: simple sampling of the exact energy
 * distribution): g[m] = number of configurations with E = -2N + 4m,
 * m = 0..N.  Written as Z = Tr T^L over rows, with integer weights in the
 * number u of unsatisfied bonds (E = -2N + 2u): a row s carries its
 * unsatisfied horizontal bonds h(s), and two neighbouring rows s, s' the
 * vertical ones, the Hamming distance of s and s'.  The Hamming factor
 * y^d(s, s') is the product over columns of (1 if equal, y if not), applied
 * one column at a time.  For each first row, the rows 2..L are added one
 * after the other and the last row is closed onto the first; polynomials in
 * y are exact 128-bit integer coefficient arrays (L <= 8).  Odd u never
 * occurs on the periodic lattice. */
typedef unsigned __int128 u128;

static int row_unsat(int s, int L)
{
    int h = 0;
    for (int x = 0; x < L; x++) h += ((s >> x) & 1) != ((s >> ((x + 1) % L)) & 1);
    return h;
}

int or_exact_dos(int L, uint64_t *out /* [N+1][2]: low, high 64 bits of g[m] */)
{
    if (L < 4 || L > 8 || (L & 1) || !out) return OR_ERR_ARG;
    const int N = L * L, U = 2 * N + 1, S = 1 << L;
    u128 *v = (u128 *)calloc((size_t)S * U, sizeof(u128));
    u128 *w = (u128 *)calloc((size_t)S * U, sizeof(u128));
    u128 *z = (u128 *)calloc((size_t)U, sizeof(u128));
    for (int s1 = 0; s1 < S; s1++) {
        memset(v, 0, sizeof(u128) * S * U);
        v[(size_t)s1 * U + row_unsat(s1, L)] = 1;
        for (int r = 1; r <= L; r++) {
            /* vertical bonds to the next row (for r = L: back to row 1) */
            for (int b = 0; b < L; b++) {
                for (int s = 0; s < S; s++)
                    for (int u = 0; u < U; u++) {
                        u128 a = v[(size_t)s * U + u];
                        if (u > 0) a += v[(size_t)(s ^ (1 << b)) * U + u - 1];
                        w[(size_t)s * U + u] = a;
                    }
                u128 *t = v; v = w; w = t;
            }
            if (r == L) break;
            /* the new row's horizontal bonds */
            for (int s = 0; s < S; s++) {
                int h = row_unsat(s, L);
                for (int u = U - 1; u >= 0; u--) v[(size_t)s * U + u] = u >= h ? v[(size_t)s * U + u - h] : 0;
            }
        }
        for (int u = 0; u < U; u++) z[u] += v[(size_t)s1 * U + u];   /* closed onto row 1 = s1 */
    }
    for (int m = 0; m <= N; m++) {
        out[2 * m] = (uint64_t)z[2 * m];
        out[2 * m + 1] = (uint64_t)(z[2 * m] >> 64);
    }
    free(v); free(w); free(z);
    return OR_OK;
}

/* Energy draw table at inverse temperature beta: weights
 * w_m = g_m exp(-4 beta m) (relative to the ground state) in FP64, g_m
 * rounded to the nearest double; cumulative S_m in increasing m; threshold
 * C_m = floor(2^64 S_m / S_N), or 2^64 - 1 where S_m / S_N = 1.  A uniform
 * 64-bit draw v selects the smallest m with v < C_m, or m = N if there is
 * none, so level m is drawn with probability w_m / S_N up to 2^-64 per
 * level. */
static void dos_table(const double *gd /* g_m rounded to the nearest double */, int N, double beta, uint64_t *C)
{
    double *S = (double *)malloc(sizeof(double) * (N + 1));
    double acc = 0.0;
    for (int m = 0; m <= N; m++) {
        acc += gd[m] * exp(-4.0 * beta * (double)m);
        S[m] = acc;
    }
    for (int m = 0; m <= N; m++) {
        double q = S[m] / acc;
        C[m] = q >= 1.0 ? UINT64_MAX : (uint64_t)ldexp(q, 64);
    }
    free(S);
}

/* The density of states of a theta = infinity run, g_m rounded to the
 * nearest double (m = 0..N): builds the energy draw tables of every
 * temperature.  Needed before the first step for L > 8. */
int or_set_dos(or_run *run, const double *gd)
{
    if (!run || !gd || run->d.theta != -1) return OR_ERR_ARG;
    const int N = run->N;
    free(run->dosC);
    run->dosC = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)run->d.K * (N + 1));
    for (int k = 0; k < run->d.K; k++) dos_table(gd, N, run->beta[k], &run->dosC[(size_t)k * (N + 1)]);
    return OR_OK;
}

/* Step (iv) at theta = infinity: every replica's energy is replaced by an
 * independent draw from the exact distribution at beta_i; the draw of
 * replica j is v = o0 | o1 << 32 of Philox(seed; j, 0, i, TAG_DOS << 28 |
 * pop << 24).  The configurations are not used in this limit. */
static void dos_sample(or_run *run, int p, int i)
{
    or_pop *P = &run->pop[p];
    const int N = run->N;
    const uint64_t *C = &run->dosC[(size_t)i * (N + 1)];
    for (int j = 0; j < P->Rcur; j++) {
        uint32_t o[4];
        philox_at(run->key, (uint32_t)j, 0, (uint32_t)i, (TAG_DOS << 28) | ((uint32_t)p << 24), o);
        uint64_t v = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        int m = N;
        for (int k = 0; k <= N; k++)
            if (v < C[k]) { m = k; break; }
        P->E[P->cur][j] = -2 * N + 4 * m;
    }
}

/* Step (i): draw R_0 = R configurations from the uniform distribution at
 * beta_0 = 0 (Sec. II A).  Replica j = 64g + b of population pi takes, at
 * site n, the spin -1 if bit b of the 64-bit word o0 | o1 << 32 of
 * Philox(seed; n, g, 0, TAG_INIT << 28 | pi << 24) is set, else +1.
 * Family labels f_j = j.  Then measure at i = 0. */
or_run *or_create(const or_desc *d)
{
    if (!d || d->L < 4 || (d->L & 1) || d->L > 1024 || d->R < 1 || d->R_cap < d->R ||
        d->theta < -1 || d->K < 2 || !d->beta || d->model < 0 || d->model > 1 ||
        d->resampling < 0 || d->resampling > 1 || d->overlap < 0 || d->overlap > 4 ||
        d->R_cap >= (1 << 23))
        return NULL;
    if (d->resampling == 0 && d->R_cap != d->R) return NULL;
    if (d->theta == -1 && (d->model != 0 || d->L > 30 || d->overlap != 0)) return NULL;
    or_run *run = (or_run *)calloc(1, sizeof(or_run));
    run->d = *d;
    run->N = d->L * d->L;
    run->npop = d->overlap == 2 ? 2 : 1;
    run->beta = (double *)malloc(sizeof(double) * d->K);
    memcpy(run->beta, d->beta, sizeof(double) * d->K);
    run->d.beta = run->beta;
    key_of(d->seed, run->key);
    int N = run->N, L = d->L;

    /* couplings: J_R(n), J_D(n) = -1 iff bit 0 (resp. bit 1) of o0 (resp. o1)
     * of Philox(disorder_seed; n, 0, 0, TAG_J << 28) is set (spin glass). */
    run->jR = (int8_t *)malloc(N);
    run->jD = (int8_t *)malloc(N);
    uint32_t dkey[2];
    key_of(d->disorder_seed, dkey);
    for (int n = 0; n < N; n++) {
        if (d->model == 1) {
            uint32_t o[4];
            philox_at(dkey, (uint32_t)n, 0, 0, TAG_J << 28, o);
            run->jR[n] = (o[0] & 1u) ? -1 : 1;
            run->jD[n] = (o[1] & 1u) ? -1 : 1;
        } else {
            run->jR[n] = 1;
            run->jD[n] = 1;
        }
    }
    (void)L;

    for (int p = 0; p < run->npop; p++) {
        or_pop *P = &run->pop[p];
        for (int b = 0; b < 2; b++) {
            P->s[b] = (int8_t *)calloc((size_t)d->R_cap * N, 1);
            P->E[b] = (int32_t *)calloc(d->R_cap, sizeof(int32_t));
            P->f[b] = (int32_t *)calloc(d->R_cap, sizeof(int32_t));
        }
        P->r = (int32_t *)calloc(d->R_cap, sizeof(int32_t));
        P->X = (uint64_t *)calloc(d->R_cap, sizeof(uint64_t));
        P->cur = 0;
        P->Rcur = d->R;
        P->Rprev = d->R;
        P->status = OR_OK;
        P->A = (double)N * log(2.0);   /* ln Z(0) = N ln 2 */
        P->lnQ = 0.0;
        for (int n = 0; n < N; n++) {
            for (int g = 0; g * 64 < d->R; g++) {
                uint32_t o[4];
                philox_at(run->key, (uint32_t)n, (uint32_t)g, 0,
                          (TAG_INIT << 28) | ((uint32_t)p << 24), o);
                uint64_t plane = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
                for (int b = 0; b < 64 && g * 64 + b < d->R; b++) {
                    int j = g * 64 + b;
                    P->s[0][(size_t)j * N + n] = ((plane >> b) & 1u) ? -1 : 1;
                }
            }
        }
        for (int j = 0; j < d->R; j++) {
            P->f[0][j] = j;
            P->E[0][j] = energy_of(run, &P->s[0][(size_t)j * N]);
        }
    }
    run->obs = (or_obs *)calloc((size_t)run->npop * d->K, sizeof(or_obs));
    if (d->theta == -1 && L <= 8) {
        /* L <= 8: the density of states of the transfer matrix above;
         * larger L: supplied with or_set_dos before the first step */
        uint64_t *g2 = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (N + 1));
        double *gd = (double *)malloc(sizeof(double) * (N + 1));
        or_exact_dos(L, g2);
        for (int m = 0; m <= N; m++) gd[m] = (double)(((u128)g2[2 * m + 1] << 64) | g2[2 * m]);
        or_set_dos(run, gd);
        free(g2); free(gd);
    }
    run->rho = (double *)malloc(sizeof(double) * run->npop * d->K);
    for (int k = 0; k < run->npop * d->K; k++) run->rho[k] = NAN;
    if (d->qhist)
        run->qh = (int32_t *)calloc((size_t)run->npop * d->K * (N + 1), sizeof(int32_t));
    run->i = 0;
    measure_impl(run, 0);
    run->phase = PH_MEASURED;
    return run;
}

/* ---------------------------------------------------- step (ii): reweight -- */

/* Q_i = (1/R_{i-1}) sum_j exp[-(beta_i - beta_{i-1}) E_j], Eq. (QBoltz),
 * evaluated relative to E_min so every term is <= 1:
 *   ln Q_i = ln( sum_j x_j ) - ln R_{i-1} - dbeta E_min,
 * and A_i = A_{i-1} + ln Q_i, Eq. (F).  The integer images X_j of x_j are
 * kept for resampling (tau_j = R X_j / sum X, Eq. (tauBoltz), in which the
 * factors R_{i-1} cancel). */
int or_anneal_step(or_run *run, int i)
{
    if (!run) return OR_ERR_ARG;
    if (run->phase != PH_MEASURED || i != run->i + 1 || i >= run->d.K) return OR_ERR_STATE;
    double dbeta = run->beta[i] - run->beta[i - 1];
    for (int p = 0; p < run->npop; p++) {
        or_pop *P = &run->pop[p];
        if (P->status != OR_OK) continue;
        const int32_t *E = P->E[P->cur];
        int32_t Rp = P->Rcur;
        int32_t Emin = E[0];
        for (int j = 1; j < Rp; j++) if (E[j] < Emin) Emin = E[j];
        double S = 0.0;
        uint64_t SX = 0;
        for (int j = 0; j < Rp; j++) {
            int k = (E[j] - Emin) / 4;
            S += or_reweight_x(dbeta, k);
            P->X[j] = or_reweight_X(dbeta, k);
            SX += P->X[j];
        }
        P->Rprev = Rp;
        P->SX = SX;
        P->lnQ = log(S) - log((double)Rp) - dbeta * (double)Emin;
        P->A += P->lnQ;
    }
    run->i = i;
    run->phase = PH_ANNEALED;
    return OR_OK;
}

/* --------------------------------------------------- step (iii): resample -- */

static void freeze(or_run *run, int p, int i, int32_t status)
{
    run->pop[p].status = status;
    for (int k = i; k < run->d.K; k++) obs_frozen(&run->obs[p * run->d.K + k], status);
}

/* Nearest-integer resampling (Sec. II B): r_j = ceil(tau_j) with probability
 * tau_j - floor(tau_j), else floor(tau_j).  tau_j = R X_j / S_X is handled as
 * the exact rational: n_j = floor(R X_j / S_X) and the fractional part as the
 * 32-bit fixed-point t_j = floor(((R X_j) mod S_X) 2^32 / S_X); with
 * u_j = o0 of Philox(seed; j, 0, i, TAG_NI << 28 | pi << 24), r_j = n_j + [u_j < t_j].
 *
 * Multinomial resampling (Sec. IV C, condition (c)): R independent draws of a
 * parent with probability X_j / S_X: draw d takes v = o0 | o1 << 32 of
 * Philox(seed; d, 0, i, TAG_MN << 28 | pi << 24), the target
 * t = floor(v S_X / 2^64), and the parent is the largest j whose exclusive
 * prefix sum P_j of X is <= t.
 *
 * The r_j copies of replica j go to the consecutive child slots
 * [C_j, C_j + r_j), C the exclusive prefix of r, so families stay contiguous
 * (Sec. V A 1).  Spins, energies and family labels are copied. */
int or_resample(or_run *run, int i)
{
    if (!run) return OR_ERR_ARG;
    if (run->phase != PH_ANNEALED || i != run->i) return OR_ERR_STATE;
    int N = run->N;
    for (int p = 0; p < run->npop; p++) {
        or_pop *P = &run->pop[p];
        if (P->status != OR_OK) continue;
        int32_t Rp = P->Rprev;
        uint64_t SX = P->SX;
        int64_t Ri = 0;
        if (run->d.resampling == 1) {
            for (int j = 0; j < Rp; j++) {
                uint64_t RX = (uint64_t)run->d.R * P->X[j];
                uint64_t nj = RX / SX;
                uint64_t rem = RX % SX;
                uint32_t tj = (uint32_t)(((unsigned __int128)rem << 32) / SX);
                uint32_t o[4];
                philox_at(run->key, (uint32_t)j, 0, (uint32_t)i,
                          (TAG_NI << 28) | ((uint32_t)p << 24), o);
                P->r[j] = (int32_t)nj + (o[0] < tj ? 1 : 0);
                Ri += P->r[j];
            }
        } else {
            uint64_t *pre = (uint64_t *)malloc(sizeof(uint64_t) * (Rp + 1));
            pre[0] = 0;
            for (int j = 0; j < Rp; j++) pre[j + 1] = pre[j] + P->X[j];
            memset(P->r, 0, sizeof(int32_t) * Rp);
            for (int dd = 0; dd < run->d.R; dd++) {
                uint32_t o[4];
                philox_at(run->key, (uint32_t)dd, 0, (uint32_t)i,
                          (TAG_MN << 28) | ((uint32_t)p << 24), o);
                uint64_t v = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
                uint64_t t = (uint64_t)(((unsigned __int128)v * SX) >> 64);
                int lo = 0, hi = Rp - 1;        /* largest j with pre[j] <= t */
                while (lo < hi) {
                    int mid = lo + (hi - lo + 1) / 2;
                    if (pre[mid] <= t) lo = mid; else hi = mid - 1;
                }
                P->r[lo]++;
            }
            free(pre);
            Ri = run->d.R;
        }
        if (Ri > run->d.R_cap) { freeze(run, p, i, OR_ERR_CAPACITY); continue; }
        if (Ri == 0) { freeze(run, p, i, OR_ERR_NUMERIC); continue; }
        int src = P->cur, dst = 1 - P->cur;
        int64_t c = 0;
        for (int j = 0; j < Rp; j++) {
            for (int k = 0; k < P->r[j]; k++, c++) {
                memcpy(&P->s[dst][(size_t)c * N], &P->s[src][(size_t)j * N], N);
                P->E[dst][c] = P->E[src][j];
                P->f[dst][c] = P->f[src][j];
            }
        }
        P->cur = dst;
        P->Rcur = (int32_t)Ri;
    }
    run->phase = PH_RESAMPLED;
    return OR_OK;
}

/* ------------------------------------------------------ step (iv): sweeps -- */

/* The 32-bit Metropolis draw of replica j = 64g + b at site n, sweep s,
 * temperature i, population pi.  It is assembled from 32 bit planes, most
 * significant first: Philox call c in [0,16) with counter
 * (n | c << 20, g, i, TAG_SWEEP << 28 | pi << 24 | s) yields plane 2c from
 * o0 | o1 << 32 and plane 2c+1 from o2 | o3 << 32; bit b of plane p is bit
 * 31-p of u_j.  The planes for all 64 lanes of a group come from the same
 * calls, so they are generated once per (site, group). */
static void sweep_planes(const uint32_t key[2], int n, int g, int i, int pop, int s,
                         uint64_t planes[32])
{
    for (int c = 0; c < 16; c++) {
        uint32_t o[4];
        philox_at(key, (uint32_t)n | ((uint32_t)c << 20), (uint32_t)g, (uint32_t)i,
                  (TAG_SWEEP << 28) | ((uint32_t)pop << 24) | (uint32_t)s, o);
        planes[2 * c] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        planes[2 * c + 1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    }
}

static uint32_t draw_from_planes(const uint64_t planes[32], int b)
{
    uint32_t u = 0;
    for (int p = 0; p < 32; p++) u |= (uint32_t)((planes[p] >> b) & 1u) << (31 - p);
    return u;
}

uint32_t or_sweep_draw(uint64_t seed, int n, int j, int i, int pop, int s)
{
    uint32_t key[2];
    uint64_t planes[32];
    key_of(seed, key);
    sweep_planes(key, n, j / 64, i, pop, s, planes);
    return draw_from_planes(planes, j % 64);
}

/* theta sweeps at beta_i.  One sweep visits colour 0 ((x + y) even) and then
 * colour 1; within a colour every site of that colour of every replica is
 * updated (sites of one colour are never neighbours for even L, so their
 * order does not matter).  Single-spin-flip Metropolis: with
 * h = sum of J s over the 4 neighbours, dE = 2 s_n h; flip if dE <= 0, else
 * flip iff u < T(beta_i, dE).  Replicas never interact during the sweeps, so
 * the 64-replica groups are processed one after the other. */
static void sweep_group(or_run *run, int p, int i, int g, uint64_t T4, uint64_t T8)
{
    int L = run->d.L, N = run->N;
    or_pop *P = &run->pop[p];
    int8_t *S = P->s[P->cur];
    int32_t *E = P->E[P->cur];
    int32_t Ri = P->Rcur;
    uint64_t planes[32];
    for (int s = 0; s < run->d.theta; s++) {
        for (int colour = 0; colour < 2; colour++) {
            for (int n = 0; n < N; n++) {
                int x = n % L, y = n / L;
                if (((x + y) & 1) != colour) continue;
                int nr = right_of(n, L), nl = left_of(n, L);
                int nd = down_of(n, L), nu = up_of(n, L);
                sweep_planes(run->key, n, g, i, p, s, planes);
                for (int b = 0; b < 64 && g * 64 + b < Ri; b++) {
                    int j = g * 64 + b;
                    int8_t *sj = &S[(size_t)j * N];
                    int h = run->jR[n] * sj[nr] + run->jR[nl] * sj[nl] +
                            run->jD[n] * sj[nd] + run->jD[nu] * sj[nu];
                    int dE = 2 * sj[n] * h;
                    int flip;
                    if (dE <= 0) {
                        flip = 1;
                    } else {
                        uint32_t u = draw_from_planes(planes, b);
                        flip = (uint64_t)u < (dE == 4 ? T4 : T8);
                    }
                    if (flip) {
                        sj[n] = (int8_t)-sj[n];
                        E[j] += dE;
                    }
                }
            }
        }
    }
}

int or_sweep(or_run *run, int i)
{
    if (!run) return OR_ERR_ARG;
    if (run->phase != PH_RESAMPLED || i != run->i) return OR_ERR_STATE;
    uint64_t T4 = or_sweep_threshold(run->beta[i], 4);
    uint64_t T8 = or_sweep_threshold(run->beta[i], 8);
    for (int p = 0; p < run->npop; p++) {
        if (run->pop[p].status != OR_OK) continue;
        if (run->d.theta == -1) {
            if (!run->dosC) return OR_ERR_STATE;   /* no density of states supplied */
            dos_sample(run, p, i);
            continue;
        }
        for (int g = 0; g * 64 < run->pop[p].Rcur; g++) sweep_group(run, p, i, g, T4, T8);
    }
    run->phase = PH_SWEPT;
    return OR_OK;
}

/* Step (iv) for a sample of replica groups only (the other replicas are
 * left as they were, so the run must not be continued afterwards).  Lets a
 * test compare sampled outputs of configurations too large to sweep whole. */
int or_sweep_groups(or_run *run, int i, const int32_t *groups, int ngroups)
{
    if (!run) return OR_ERR_ARG;
    if (run->phase != PH_RESAMPLED || i != run->i) return OR_ERR_STATE;
    uint64_t T4 = or_sweep_threshold(run->beta[i], 4);
    uint64_t T8 = or_sweep_threshold(run->beta[i], 8);
    for (int p = 0; p < run->npop; p++) {
        if (run->pop[p].status != OR_OK) continue;
        for (int k = 0; k < ngroups; k++)
            if (groups[k] >= 0 && groups[k] * 64 < run->pop[p].Rcur)
                sweep_group(run, p, i, groups[k], T4, T8);
    }
    run->phase = PH_SWEPT;
    return OR_OK;
}

/* ----------------------------------------------------- step (v): measure -- */

/* Integer sums over the population at beta_i: sum E, sum E^2, sum |M|,
 * sum M^2 (Eqs. (e), (m) and the squared-summand averages behind (c), (chi));
 * spin overlaps Q = N q = sum_n s_n s'_n for the index-shift pairs
 * (j, j + floor(R_i/2)), j < floor(R_i/2) (Sec. III D), for the pairs
 * (j of population 0, j of population 1), j < min(R_0, R_1), or for the R_i
 * pairs (k, pi_k) of the permutation pairing below; link overlaps
 * Q_l = sum over the 2N bonds of (s_m s_n)(s'_m s'_n); family sizes c_f. */
static void pair_overlap(const or_run *run, const int8_t *a, const int8_t *b,
                         int64_t *Q, int64_t *Ql, int *ham)
{
    int L = run->d.L, N = run->N;
    int64_t q = 0, ql = 0;
    int h = 0;
    for (int n = 0; n < N; n++) {
        q += a[n] * b[n];
        h += a[n] != b[n];
        int r = right_of(n, L), d = down_of(n, L);
        ql += (a[n] * a[r]) * (b[n] * b[r]);
        ql += (a[n] * a[d]) * (b[n] * b[d]);
    }
    *Q = q; *Ql = ql; *ham = h;
}

static void add_pair(or_obs *o, int32_t *hist, int64_t Q, int64_t Ql, int ham)
{
    o->nPairs++;
    o->sumQ += Q;
    o->sumAbsQ += Q < 0 ? -Q : Q;
    o->sumQ2 += Q * Q;
    o->sumQl += Ql;
    o->sumQl2 += Ql * Ql;
    if (hist) hist[ham]++;
}

/* ------------------------------------------- permutation pairing (q) -- */

/* A uniformly random permutation of [0, R) for the pairing at temperature
 * i of population pop: position m holds the index with the m-th smallest
 * 64-bit key, ties by index.  The key of index k is o0 | o1 << 32
 * (which = 0, the initial permutation pi) or o2 | o3 << 32 (which = 1, the
 * search pattern sigma) of Philox(seed; k, 0, i, TAG_PERM << 28 | pop << 24). */
typedef struct { uint64_t key; int32_t idx; } keyed;

static int keyed_cmp(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

int or_random_permutation(uint64_t seed, int i, int pop, int R, int which, int32_t *out)
{
    if (R < 0 || (which != 0 && which != 1) || (R > 0 && !out)) return OR_ERR_ARG;
    uint32_t key[2];
    key_of(seed, key);
    keyed *k = (keyed *)malloc(sizeof(keyed) * (R > 0 ? R : 1));
    for (int j = 0; j < R; j++) {
        uint32_t o[4];
        philox_at(key, (uint32_t)j, 0, (uint32_t)i, (TAG_PERM << 28) | ((uint32_t)pop << 24), o);
        k[j].key = which == 0 ? ((uint64_t)o[0] | ((uint64_t)o[1] << 32))
                              : ((uint64_t)o[2] | ((uint64_t)o[3] << 32));
        k[j].idx = j;
    }
    qsort(k, R, sizeof(keyed), keyed_cmp);
    for (int m = 0; m < R; m++) out[m] = k[m].idx;
    free(k);
    return OR_OK;
}

/* Size of the largest family among labels fam[0..R). */
static int32_t largest_family(const int32_t *fam, int R)
{
    int32_t mx = 0, lab = 0;
    for (int j = 0; j < R; j++)
        if (fam[j] > lab) lab = fam[j];
    int32_t *c = (int32_t *)calloc((size_t)lab + 1, sizeof(int32_t));
    for (int j = 0; j < R; j++)
        if (++c[fam[j]] > mx) mx = c[fam[j]];
    free(c);
    return mx;
}

/* Sec. III D, pairings from permutations (Wang et al.): turns the
 * permutation pi (in place) into one in which no position k is paired with
 * a replica of its own family, fam[pi[k]] != fam[k]; the overlaps are then
 * those of the R pairs (k, pi[k]), every replica used twice.
 *   sigma == NULL: repeatedly take the smallest position k whose pair is
 *   incestuous and walk l = 1, 2, ... (positions mod R) to the first k + l
 *   with pi[k + l] outside k's family and pi[k] outside the family of k + l;
 *   exchange pi[k] and pi[k + l].
 *   sigma != NULL (random search pattern): go through the positions in the
 *   order sigma[0], sigma[1], ...; a mismatch at k = sigma[t] is repaired
 *   with the first sigma[t + l], l = 1, 2, ... (indices of sigma mod R),
 *   under the same two conditions.
 * An exchange leaves both of its positions matched and touches no other, so
 * the number of mismatches falls by at least one each time.  A suitable
 * partner exists whenever no family holds more than R/2 replicas; if one
 * does, no such permutation exists at all, pi is left as it was and 1 is
 * returned (the measurement is then omitted).  Parity: pinned by brute
 * force on small populations (tests). */
int or_wang_repair(const int32_t *fam, int R, int32_t *pi, const int32_t *sigma)
{
    if (R < 1 || !fam || !pi) return OR_ERR_ARG;
    if (2 * (int64_t)largest_family(fam, R) > R) return 1;
    if (!sigma) {
        for (;;) {
            int k = -1;
            for (int j = 0; j < R && k < 0; j++)
                if (fam[pi[j]] == fam[j]) k = j;
            if (k < 0) return OR_OK;
            int found = 0;
            for (int l = 1; l < R && !found; l++) {
                int m = (k + l) % R;
                if (fam[pi[m]] != fam[k] && fam[pi[k]] != fam[m]) {
                    int32_t t = pi[k]; pi[k] = pi[m]; pi[m] = t;
                    found = 1;
                }
            }
            if (!found) return OR_ERR_NUMERIC;   /* unreachable when no family exceeds R/2 */
        }
    }
    for (int t = 0; t < R; t++) {
        int k = sigma[t];
        if (fam[pi[k]] != fam[k]) continue;
        int found = 0;
        for (int l = 1; l < R && !found; l++) {
            int m = sigma[(t + l) % R];
            if (fam[pi[m]] != fam[k] && fam[pi[k]] != fam[m]) {
                int32_t x = pi[k]; pi[k] = pi[m]; pi[m] = x;
                found = 1;
            }
        }
        if (!found) return OR_ERR_NUMERIC;
    }
    return OR_OK;
}

/* The pairing of population p at temperature i for overlap kinds 3 and 4:
 * pi from or_random_permutation, repaired by or_wang_repair (with sigma for
 * kind 4).  Returns 0 and fills out[R_i], or 1 when a family is too large. */
static int wang_pairing(const or_run *run, int p, int i, int32_t *out)
{
    const or_pop *P = &run->pop[p];
    int R = P->Rcur;
    or_random_permutation(run->d.seed, i, p, R, 0, out);
    int32_t *sigma = NULL;
    if (run->d.overlap == 4) {
        sigma = (int32_t *)malloc(sizeof(int32_t) * R);
        or_random_permutation(run->d.seed, i, p, R, 1, sigma);
    }
    int st = or_wang_repair(P->f[P->cur], R, out, sigma);
    free(sigma);
    return st;
}

/* The repaired pairing of population p as it stands (for tests): returns 0
 * and fills out[R_i], 1 if a family holds more than R_i/2 replicas, or an
 * error for a run without permutation pairing. */
int or_get_pairing(const or_run *run, int p, int32_t *out)
{
    if (!run || p < 0 || p >= run->npop || !out || run->d.overlap < 3) return OR_ERR_ARG;
    return wang_pairing(run, p, run->i, out);
}

static int measure_impl(or_run *run, int i)
{
    int N = run->N, K = run->d.K;
    for (int p = 0; p < run->npop; p++) {
        or_pop *P = &run->pop[p];
        if (P->status != OR_OK) continue;
        or_obs *o = &run->obs[p * K + i];
        memset(o, 0, sizeof(*o));
        const int8_t *S = P->s[P->cur];
        int32_t *E = P->E[P->cur];
        const int32_t *F = P->f[P->cur];
        int32_t Ri = P->Rcur;
        o->R_i = Ri;
        o->lnQ = i == 0 ? 0.0 : P->lnQ;
        o->A = P->A;
        int32_t Emin = 0;
        for (int j = 0; j < Ri; j++) {
            const int8_t *sj = &S[(size_t)j * N];
            if (run->d.theta == -1) {   /* energies only (theta = infinity) */
                int32_t e = i == 0 ? energy_of(run, sj) : E[j];
                E[j] = e;
                o->sumE += e;
                o->sumE2 += (int64_t)e * e;
                if (j == 0 || e < Emin) Emin = e;
                continue;
            }
            int32_t e = energy_of(run, sj);
            if (e != E[j]) run->e_mismatch++;
            E[j] = e;
            int32_t M = magnetisation_of(run, sj);
            o->sumE += e;
            o->sumE2 += (int64_t)e * e;
            o->sumAbsM += M < 0 ? -M : M;
            o->sumM2 += (int64_t)M * M;
            if (j == 0 || e < Emin) Emin = e;
        }
        o->Emin = Emin;
        P->Emin = Emin;
        int32_t *counts = (int32_t *)calloc(run->d.R, sizeof(int32_t));
        for (int j = 0; j < Ri; j++) counts[F[j]]++;
        double rho = 0.0;   /* Eq. (rho_t): R_i sum_k n_k^2, n_k = c_k / R_i */
        for (int f = 0; f < run->d.R; f++) {
            int64_t c = counts[f];
            o->famSumSq += c * c;
            if (c > o->famMax) o->famMax = c;
            if (c > 0) o->nFam++;
            if (c > 0) {
                double n = (double)c / (double)Ri;
                rho += n * n;
            }
        }
        run->rho[(size_t)p * K + i] = (double)Ri * rho;
        free(counts);
        int32_t *hist = run->qh ? &run->qh[((size_t)p * K + i) * (N + 1)] : NULL;
        if (hist) memset(hist, 0, sizeof(int32_t) * (N + 1));
        if (run->d.overlap == 1) {
            int h = Ri / 2;
            for (int j = 0; j < h; j++) {
                int64_t Q, Ql;
                int ham;
                pair_overlap(run, &S[(size_t)j * N], &S[(size_t)(j + h) * N], &Q, &Ql, &ham);
                add_pair(o, hist, Q, Ql, ham);
            }
        } else if (run->d.overlap >= 3) {
            int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * Ri);
            if (wang_pairing(run, p, i, pi) == OR_OK)
                for (int k = 0; k < Ri; k++) {
                    int64_t Q, Ql;
                    int ham;
                    pair_overlap(run, &S[(size_t)k * N], &S[(size_t)pi[k] * N], &Q, &Ql, &ham);
                    add_pair(o, hist, Q, Ql, ham);
                }
            free(pi);
        }
        o->status = OR_OK;
    }
    if (run->d.overlap == 2 && run->pop[0].status == OR_OK && run->pop[1].status == OR_OK) {
        or_pop *A = &run->pop[0], *B = &run->pop[1];
        or_obs *oa = &run->obs[0 * K + i], *ob = &run->obs[1 * K + i];
        int32_t *ha = run->qh ? &run->qh[((size_t)0 * K + i) * (N + 1)] : NULL;
        int32_t *hb = run->qh ? &run->qh[((size_t)1 * K + i) * (N + 1)] : NULL;
        int m = A->Rcur < B->Rcur ? A->Rcur : B->Rcur;
        for (int j = 0; j < m; j++) {
            int64_t Q, Ql;
            int ham;
            pair_overlap(run, &A->s[A->cur][(size_t)j * N], &B->s[B->cur][(size_t)j * N],
                         &Q, &Ql, &ham);
            add_pair(oa, ha, Q, Ql, ham);
            add_pair(ob, hb, Q, Ql, ham);
        }
    }
    return OR_OK;
}

int or_measure(or_run *run, int i)
{
    if (!run) return OR_ERR_ARG;
    if (run->phase != PH_SWEPT || i != run->i) return OR_ERR_STATE;
    measure_impl(run, i);
    run->phase = PH_MEASURED;
    return OR_OK;
}

/* All K-1 temperature steps (ii)-(v) in order. */
int or_anneal_all(or_run *run)
{
    for (int i = run->i + 1; i < run->d.K; i++) {
        int st;
        if ((st = or_anneal_step(run, i))) return st;
        if ((st = or_resample(run, i))) return st;
        if ((st = or_sweep(run, i))) return st;
        if ((st = or_measure(run, i))) return st;
    }
    return OR_OK;
}

/* ------------------------------------------------------------- accessors -- */

int or_get_info(const or_run *run, int32_t *out /* [6]: i, phase, N, npop, K, R */)
{
    out[0] = run->i; out[1] = run->phase; out[2] = run->N;
    out[3] = run->npop; out[4] = run->d.K; out[5] = run->d.R;
    return OR_OK;
}

int64_t or_energy_mismatches(const or_run *run) { return run->e_mismatch; }

/* Current population of population p: spins [R_i][N] (+1/-1), energies,
 * family labels; returns R_i (or -1 on a bad argument). */
int32_t or_get_state(const or_run *run, int p, int8_t *spins, int32_t *E, int32_t *fam,
                     int32_t *status)
{
    if (p < 0 || p >= run->npop) return -1;
    const or_pop *P = &run->pop[p];
    int32_t Ri = P->Rcur;
    if (spins) memcpy(spins, P->s[P->cur], (size_t)Ri * run->N);
    if (E) memcpy(E, P->E[P->cur], sizeof(int32_t) * Ri);
    if (fam) memcpy(fam, P->f[P->cur], sizeof(int32_t) * Ri);
    if (status) *status = P->status;
    return Ri;
}

/* Descendant counts of the last resampling of population p; returns the
 * parent population size R_{i-1}. */
int32_t or_get_counts(const or_run *run, int p, int32_t *r, uint64_t *X, uint64_t *SX)
{
    if (p < 0 || p >= run->npop) return -1;
    const or_pop *P = &run->pop[p];
    if (r) memcpy(r, P->r, sizeof(int32_t) * P->Rprev);
    if (X) memcpy(X, P->X, sizeof(uint64_t) * P->Rprev);
    if (SX) *SX = P->SX;
    return P->Rprev;
}

int or_get_couplings(const or_run *run, int8_t *jR, int8_t *jD)
{
    memcpy(jR, run->jR, run->N);
    memcpy(jD, run->jD, run->N);
    return OR_OK;
}

int or_get_obs(const or_run *run, or_obs *out /* [npop][K] */)
{
    memcpy(out, run->obs, sizeof(or_obs) * run->npop * run->d.K);
    return OR_OK;
}

int or_get_qhist(const or_run *run, int32_t *out /* [npop][K][N+1] */)
{
    if (!run->qh) return OR_ERR_ARG;
    memcpy(out, run->qh, sizeof(int32_t) * run->npop * run->d.K * (run->N + 1));
    return OR_OK;
}

int or_get_rho(const or_run *run, double *out /* [npop][K] */)
{
    memcpy(out, run->rho, sizeof(double) * run->npop * run->d.K);
    return OR_OK;
}

/* ------------------------------------------------------ weighted average -- */

/* Per-run estimators at temperature i from the integer sums of one record. */
typedef struct { double e, e2, c, m, m2, chi, absq, q2, ql; } run_est;

static run_est estimators(const or_obs *o, double beta, int N)
{
    run_est r;
    double Ri = (double)o->R_i, dN = (double)N;
    __int128 varE = (__int128)o->R_i * o->sumE2 - (__int128)o->sumE * o->sumE;
    __int128 varM = (__int128)o->R_i * o->sumM2 - (__int128)o->sumAbsM * o->sumAbsM;
    r.e = (double)o->sumE / (dN * Ri);
    r.e2 = (double)o->sumE2 / (dN * dN * Ri);
    r.c = beta * beta * (double)varE / (dN * Ri * Ri);           /* Eq. (c) */
    r.m = (double)o->sumAbsM / (dN * Ri);
    r.m2 = (double)o->sumM2 / (dN * dN * Ri);
    r.chi = beta * (double)varM / (dN * Ri * Ri);                 /* Eq. (chi) */
    if (o->nPairs > 0) {
        double np = (double)o->nPairs;
        r.absq = (double)o->sumAbsQ / (dN * np);
        r.q2 = (double)o->sumQ2 / (dN * dN * np);
        r.ql = (double)o->sumQl / (2.0 * dN * np);
    } else {
        r.absq = r.q2 = r.ql = 0.0;
    }
    return r;
}

/* Log of the unnormalised free-energy weight of run m at temperature i:
 * simplified, Eq. (simpleWeight): ln R_i + A_i;
 * full, Eq. (appropriateWeight): ln R_i + sum_{k=1..i} ln(R_{k-1}/R) + A_i. */
static double log_weight(const or_obs *om /* [K] of run m */, int i, int kind, int32_t R)
{
    double a = log((double)om[i].R_i) + om[i].A;
    if (kind == 0)
        for (int k = 1; k <= i; k++) a += log((double)om[k - 1].R_i / (double)R);
    return a;
}

/* The log-weights a[m][i] that the weighted averages use (log_weight above),
 * NaN for records whose status is not OK; kind as in or_weighted_average
 * (bit 0: simplified).  Exported so that the tests can check the weights
 * themselves: for the full weight, exp(a - ln R - N ln 2) is an unbiased
 * estimate of Z(beta_i)/2^N (the population-size argument of Sec. IV A). */
int or_log_weights(const or_obs *obs, int M, int K, const int32_t *R, int kind, double *out /* [M][K] */)
{
    if (M < 1 || K < 1 || !obs || !R || !out || kind < 0 || kind > 3) return OR_ERR_ARG;
    for (int m = 0; m < M; m++)
        for (int i = 0; i < K; i++) {
            const or_obs *om = &obs[(size_t)m * K];
            out[(size_t)m * K + i] = om[i].status == OR_OK ? log_weight(om, i, kind & 1, R[m]) : NAN;
        }
    return OR_OK;
}

/* Weighted averages over M runs (Sec. IV), for each temperature i.
 * obs: [M][K] records of one population of each run; R: target size per run;
 * kind: 0 = full weight, 1 = simplified weight.  Runs whose record has a
 * non-OK status are left out; n_included counts the others.
 * W[O] = sum_m w_m O_m, Eq. (W_conf); W_var[c] = beta^2 N (W[e^2] - W[e]^2),
 * Eq. (Wvar_C), evaluated through the identity of Eq. (Wvar_bound) as
 * sum w c_m + beta^2 N sum w (e_m - W[e])^2 (same for chi with m and beta);
 * -beta_i W[F_i] = ln Z(beta_0) + sum_{k<=i} ln W[Q_k], Eq. (W_F), with
 * W[Q_k] = sum_m w_{k-1}^(m) Q_k^(m) over the runs still included at k;
 * var_w = (1/n) sum (w - 1/n)^2 and var_w_pred = (exp(var A_i) - 1)/n^2,
 * Eq. (varWpred), var taken as (1/n) sum (A - mean A)^2. */
/* A family holds more than R_i / 2 replicas at temperature i in run m
 * (Sec. III D, Table I); obs_other: the other population of two-population
 * runs, or NULL. */
static int family_over_half(const or_obs *obs, const or_obs *obs_other, int K, int m, int i)
{
    const or_obs *o = &obs[(size_t)m * K + i];
    if (2 * o->famMax > o->R_i) return 1;
    if (obs_other) {
        const or_obs *q = &obs_other[(size_t)m * K + i];
        if (2 * q->famMax > q->R_i) return 1;
    }
    return 0;
}

/* Weights of the overlap averages at temperature i: w_m over the runs with
 * status OK, leaving out (flag 2 of kind) runs with a family above R_i / 2;
 * returns the number of runs kept (0: no weights). */
static int overlap_weights(const or_obs *obs, const or_obs *obs_other, int M, int K, int i, int kind,
                           const int32_t *R, double *w)
{
    double amax = -INFINITY;
    int n = 0;
    double *a = (double *)malloc(sizeof(double) * M);
    for (int m = 0; m < M; m++) {
        const or_obs *om = &obs[(size_t)m * K];
        a[m] = NAN;
        if (om[i].status != OR_OK) continue;
        if ((kind & 2) && family_over_half(obs, obs_other, K, m, i)) continue;
        a[m] = log_weight(om, i, kind & 1, R[m]);
        if (a[m] > amax) amax = a[m];
        n++;
    }
    double Z = 0.0;
    for (int m = 0; m < M; m++)
        if (!isnan(a[m])) Z += exp(a[m] - amax);
    for (int m = 0; m < M; m++) w[m] = isnan(a[m]) ? 0.0 : exp(a[m] - amax) / Z;
    free(a);
    return n;
}

int or_weighted_average(const or_obs *obs, const or_obs *obs_other, int M, int K, const double *beta, int N,
                        const int32_t *R, int kind, or_wavg *out /* [K] */)
{
    if (M < 1 || K < 1 || !obs || !beta || !R || !out || kind < 0 || kind > 3) return OR_ERR_ARG;
    double *wq = (double *)malloc(sizeof(double) * M);
    double *a = (double *)malloc(sizeof(double) * M);
    double *w = (double *)malloc(sizeof(double) * M);
    double *aprev = (double *)malloc(sizeof(double) * M);
    double mbWF = 0.0;
    for (int i = 0; i < K; i++) {
        or_wavg *o = &out[i];
        memset(o, 0, sizeof(*o));
        int n = 0;
        double amax = -INFINITY;
        for (int m = 0; m < M; m++) {
            const or_obs *om = &obs[(size_t)m * K];
            if (om[i].status != OR_OK) continue;
            a[m] = log_weight(om, i, kind & 1, R[m]);
            if (a[m] > amax) amax = a[m];
            n++;
        }
        o->n_included = n;
        if (n == 0) {
            double nan = NAN;
            o->W_e = o->W_e2 = o->Wvar_c = o->Wconf_c = o->W_m = o->W_m2 = nan;
            o->Wvar_chi = o->Wconf_chi = o->W_absq = o->W_q2 = o->W_ql = nan;
            o->minus_beta_WF = o->var_w = o->var_w_pred = nan;
            mbWF = nan;
            continue;
        }
        double Z = 0.0;
        for (int m = 0; m < M; m++)
            if (obs[(size_t)m * K + i].status == OR_OK) Z += exp(a[m] - amax);
        double b = beta[i];
        double sumA = 0.0;
        for (int m = 0; m < M; m++) {
            const or_obs *om = &obs[(size_t)m * K + i];
            if (om->status != OR_OK) continue;
            w[m] = exp(a[m] - amax) / Z;
            run_est r = estimators(om, b, N);
            o->W_e += w[m] * r.e;
            o->W_e2 += w[m] * r.e2;
            o->Wconf_c += w[m] * r.c;
            o->W_m += w[m] * r.m;
            o->W_m2 += w[m] * r.m2;
            o->Wconf_chi += w[m] * r.chi;
            sumA += om->A;
        }
        /* overlap averages, with their own weights (exclusion flag) */
        if (overlap_weights(obs, obs_other, M, K, i, kind, R, wq) == 0) {
            o->W_absq = o->W_q2 = o->W_ql = NAN;
        } else {
            for (int m = 0; m < M; m++) {
                const or_obs *om = &obs[(size_t)m * K + i];
                if (om->status != OR_OK || ((kind & 2) && family_over_half(obs, obs_other, K, m, i))) continue;
                run_est r = estimators(om, b, N);
                o->W_absq += wq[m] * r.absq;
                o->W_q2 += wq[m] * r.q2;
                o->W_ql += wq[m] * r.ql;
            }
        }
        double se = 0.0, sm = 0.0, vw = 0.0, va = 0.0;
        double meanA = sumA / n;
        for (int m = 0; m < M; m++) {
            const or_obs *om = &obs[(size_t)m * K + i];
            if (om->status != OR_OK) continue;
            run_est r = estimators(om, b, N);
            se += w[m] * (r.e - o->W_e) * (r.e - o->W_e);
            sm += w[m] * (r.m - o->W_m) * (r.m - o->W_m);
            vw += (w[m] - 1.0 / n) * (w[m] - 1.0 / n);
            va += (om->A - meanA) * (om->A - meanA);
        }
        o->Wvar_c = o->Wconf_c + b * b * (double)N * se;
        o->Wvar_chi = o->Wconf_chi + b * (double)N * sm;
        o->var_w = vw / n;
        o->var_w_pred = (exp(va / n) - 1.0) / ((double)n * n);
        if (i == 0) {
            /* ln Z(beta_0) = N ln 2, carried by every run as A_0 */
            mbWF = obs[0].A;
            for (int m = 0; m < M; m++)
                if (obs[(size_t)m * K].status == OR_OK) { mbWF = obs[(size_t)m * K].A; break; }
        } else {
            /* ln W[Q_i] = ln sum_m w_{i-1}^(m) Q_i^(m), the weights w_{i-1}
             * renormalised over the runs still included at i */
            double mx = -INFINITY, mx0 = -INFINITY;
            for (int m = 0; m < M; m++) {
                if (obs[(size_t)m * K + i].status != OR_OK) continue;
                double t = aprev[m] + obs[(size_t)m * K + i].lnQ;
                if (t > mx) mx = t;
                if (aprev[m] > mx0) mx0 = aprev[m];
            }
            double s1 = 0.0, s0 = 0.0;
            for (int m = 0; m < M; m++) {
                if (obs[(size_t)m * K + i].status != OR_OK) continue;
                s1 += exp(aprev[m] + obs[(size_t)m * K + i].lnQ - mx);
                s0 += exp(aprev[m] - mx0);
            }
            mbWF += (mx + log(s1)) - (mx0 + log(s0));
        }
        o->minus_beta_WF = mbWF;
        for (int m = 0; m < M; m++) aprev[m] = a[m];
    }
    free(a); free(w); free(aprev); free(wq);
    return OR_OK;
}

/* Eq. (W_conf_q): W[P(q)] = sum_m w^(m) P^(m)(q), P^(m) the empirical
 * distribution of run m's overlap pairs at temperature i (its histogram
 * over Hamming distances divided by its number of pairs).  qh: [M][K][N+1]
 * histograms of the weighted population; out: [K][N+1], NaN where no run is
 * kept. */
int or_weighted_qhist(const or_obs *obs, const or_obs *obs_other, const int32_t *qh, int M, int K, int N,
                      const int32_t *R, int kind, double *out)
{
    if (M < 1 || K < 1 || !obs || !qh || !R || !out || kind < 0 || kind > 3) return OR_ERR_ARG;
    double *w = (double *)malloc(sizeof(double) * M);
    for (int i = 0; i < K; i++) {
        double *o = &out[(size_t)i * (N + 1)];
        if (overlap_weights(obs, obs_other, M, K, i, kind, R, w) == 0) {
            for (int d = 0; d <= N; d++) o[d] = NAN;
            continue;
        }
        for (int d = 0; d <= N; d++) {
            double acc = 0.0;
            for (int m = 0; m < M; m++) {
                const or_obs *om = &obs[(size_t)m * K + i];
                if (w[m] == 0.0 || om->nPairs <= 0) continue;
                const int32_t h = qh[((size_t)m * K + i) * (N + 1) + d];
                acc += w[m] * ((double)h / (double)om->nPairs);
            }
            o[d] = acc;
        }
    }
    free(w);
    return OR_OK;
}

/* Family statistics per temperature of one run's population: rho_t from
 * Eq. (rho_t) (computed in the measurement from the family histogram), the
 * largest family, whether it exceeds R_i / 2, and whether the run is left
 * out of overlap averages (a large family in either population, or a status
 * other than OK). */
typedef struct {
    double rho_t;
    int32_t R_i, famMax, large, excluded;
} or_famstat;

int or_family_stats(const double *rho /* [K] */, const or_obs *obs /* [K] */, const or_obs *obs_other,
                    int K, or_famstat *out /* [K] */)
{
    for (int i = 0; i < K; i++) {
        const or_obs *o = &obs[i];
        or_famstat f = {NAN, (int32_t)o->R_i, (int32_t)o->famMax, 0, 1};
        if (o->status == OR_OK && o->R_i > 0) {
            f.rho_t = rho[i];
            f.large = 2 * o->famMax > o->R_i;
            f.excluded = family_over_half(obs, obs_other, K, 0, i);
        }
        out[i] = f;
    }
    return OR_OK;
}

/* ------------------------------------------------- many-run test harness -- */

/* Runs M independent copies of a descriptor (seed + m for run m) through all
 * K-1 steps and stores A_i (= -beta_i F_i) and the energy sums per run and
 * temperature: A[m][K], sumE[m][K], Rr[m][K].  Used by the statistical
 * (unbiasedness) tests; it only loops over or_create/or_anneal_all. */
int or_many_runs(const or_desc *d, int M, double *A, int64_t *sumE, int64_t *Rr)
{
    or_desc dd = *d;
    for (int m = 0; m < M; m++) {
        dd.seed = d->seed + (uint64_t)m;
        or_run *run = or_create(&dd);
        if (!run) return OR_ERR_ARG;
        int st = or_anneal_all(run);
        if (st) { or_destroy(run); return st; }
        for (int i = 0; i < d->K; i++) {
            const or_obs *o = &run->obs[i];
            if (A) A[(size_t)m * d->K + i] = o->status == OR_OK ? o->A : NAN;
            if (sumE) sumE[(size_t)m * d->K + i] = o->sumE;
            if (Rr) Rr[(size_t)m * d->K + i] = o->R_i;
        }
        or_destroy(run);
    }
    return OR_OK;
}

/* Same as or_many_runs, but keeps the complete per-temperature records of
 * population 0 of every run: obs[m][K]. */
int or_many_runs_obs(const or_desc *d, int M, or_obs *obs)
{
    or_desc dd = *d;
    for (int m = 0; m < M; m++) {
        dd.seed = d->seed + (uint64_t)m;
        or_run *run = or_create(&dd);
        if (!run) return OR_ERR_ARG;
        int st = or_anneal_all(run);
        if (st) { or_destroy(run); return st; }
        memcpy(&obs[(size_t)m * d->K], run->obs, sizeof(or_obs) * d->K);
        or_destroy(run);
    }
    return OR_OK;
}
