// pa_api.hip -- host implementation of the C ABI declared in include/pa.h.
//
// The context carves every device buffer out of the caller's workspace
// (nothing is allocated on the device here), computes the threshold and
// reweighting tables on the host in FP64 (no contraction, C library exp), and
// enqueues the kernels of kernels.hip on the caller's stream.  Argument and
// call-order validation precede every device call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace pa;

namespace {

constexpr uint64_t CKPT_MAGIC = 0x50414d4933353558ull;  // "PAMI355X"
constexpr uint32_t CKPT_VERSION = 2;

struct CkptHeader {
    uint64_t magic;
    uint32_t version, repr;
    uint64_t ws_used;
    int32_t n_runs, i, phase, npop_ctx;
    uint64_t desc_hash;     // of every run descriptor and schedule of the context
};

// FNV-1a over the fields of every run descriptor and its schedule: a
// checkpoint restores only into a context built from the same runs.
uint64_t descs_hash(const pa_ctx *c)
{
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&h](const void *p, size_t n) {
        const uint8_t *b = (const uint8_t *)p;
        for (size_t k = 0; k < n; ++k) {
            h ^= b[k];
            h *= 0x100000001b3ull;
        }
    };
    for (int r = 0; r < c->n_runs; ++r) {
        const pa_run_desc &d = c->descs[r];
        const int32_t ints[] = {d.L, (int32_t)d.model, d.R, d.R_cap, d.theta, d.K, (int32_t)d.resampling,
                                (int32_t)d.overlap, d.qhist};
        mix(ints, sizeof(ints));
        mix(&d.seed, sizeof(d.seed));
        mix(&d.disorder_seed, sizeof(d.disorder_seed));
        mix(c->betas[r].data(), sizeof(double) * c->betas[r].size());
    }
    return h;
}

// Device workspace owned by the library itself, for callers that cannot
// allocate device memory (pa_create_static).  Each GPU the library runs on
// holds its own copy of this array until the process ends.  In host code the
// array's name is not a device address: it is resolved once per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t STATIC_WS_BYTES = PA_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) uint8_t scratch[STATIC_WS_BYTES];

struct StaticWs {
    uint8_t *ptr = nullptr;          // this device's copy of `scratch`
    const pa_ctx *owner = nullptr;   // the live context using it, if any
};
std::mutex g_static_mu;
std::map<int, StaticWs> g_static_ws;   // device ordinal -> its array

bool same_table(const TableOff &t, int N, const pa_run_desc &d)
{
    return t.N == N && t.K == d.K && std::memcmp(t.beta_src, d.beta, sizeof(double) * d.K) == 0;
}

}  // namespace

namespace pa {

bool desc_ok(const pa_run_desc &d, pa_repr repr)
{
    if (d.L < 4 || d.L > 1024 || (d.L & 1)) return false;
    if (repr == PA_MSC64 && d.L > 128) return false;
    if (d.model != PA_FM && d.model != PA_EA_PMJ) return false;
    if (d.R < 1 || d.R_cap < d.R || d.R_cap >= (1 << 23)) return false;
    if (d.resampling != PA_MULTINOMIAL && d.resampling != PA_NEAREST_INT) return false;
    if (d.resampling == PA_MULTINOMIAL && d.R_cap != d.R) return false;
    if (d.overlap < PA_Q_NONE || d.overlap > PA_Q_WANG_RDM) return false;
    if (d.qhist != 0 && d.qhist != 1) return false;
    if (d.theta == PA_THETA_EXACT) {
        if (d.model != PA_FM || d.L > 30 || d.overlap != PA_Q_NONE) return false;
    } else if (d.theta < 0 || d.theta >= (1 << 24)) {
        return false;
    }
    if (d.K < 2 || d.K > (1 << 20) || d.beta == nullptr) return false;
    if (d.beta[0] != 0.0) return false;
    for (int i = 0; i < d.K; ++i)
        if (!std::isfinite(d.beta[i])) return false;
    // annealing cools: a step with beta_i < beta_{i-1} would make the
    // reweighting factors exp(-dbeta 4k) exceed one and overflow the 40-bit
    // fixed-point table and the integer sums built from it
    for (int i = 1; i < d.K; ++i)
        if (d.beta[i] < d.beta[i - 1]) return false;
    const double N = (double)d.L * d.L;
    if (4.0 * N * N * (double)d.R_cap >= 4.0e18) return false;  // int64 sums of E^2, Q_l^2
    return true;
}

void plan_run_buffers(Planner &P, const pa_run_desc &d, pa_repr repr, RunOff &o)
{
    std::memset(&o, 0, sizeof(o));
    const int N = d.L * d.L;
    const int npop = n_pop_of(d.overlap);
    const size_t site_bytes = repr == PA_MSC64 ? 8 : 64;
    const size_t nch = chunks_cap_of(d);
    for (int p = 0; p < npop; ++p) {
        for (int b = 0; b < 2; ++b) {
            o.spins[p][b] = P.take((size_t)groups_cap_of(d) * N * site_bytes);
            o.E[p][b] = P.take(sizeof(int32_t) * d.R_cap);
            o.fam[p][b] = P.take(sizeof(int32_t) * d.R_cap);
        }
        o.r[p] = P.take(sizeof(int32_t) * d.R_cap);
        o.C[p] = P.take(sizeof(int32_t) * (d.R_cap + 1));
        o.parent[p] = P.take(sizeof(int32_t) * d.R_cap);
        o.P[p] = d.resampling == PA_MULTINOMIAL ? P.take(sizeof(uint64_t) * (d.R_cap + 1)) : 0;
        o.part[p] = P.take(sizeof(int64_t) * MEAS_PART * groups_cap_of(d));
        o.partS[p] = P.take(sizeof(double) * nch);
        o.tot64[p] = P.take(sizeof(uint64_t) * nch);
        o.base64[p] = P.take(sizeof(uint64_t) * nch);
        o.tot32[p] = P.take(sizeof(int32_t) * nch);
        o.base32[p] = P.take(sizeof(int32_t) * nch);
    }
    o.qh = d.qhist ? P.take(sizeof(int32_t) * (size_t)npop * d.K * (N + 1)) : 0;
    o.jbits = P.take(N);
    o.wang = is_wang(d.overlap) ? P.take(sizeof(int32_t) * wang_ints(d.R_cap, N)) : 0;
    o.dos = d.theta == PA_THETA_EXACT ? P.take(sizeof(uint64_t) * (size_t)d.K * (N + 1)) : 0;
}

void plan_table(Planner &P, int N, const pa_run_desc &d, TableOff &T)
{
    T.N = N;
    T.K = d.K;
    T.beta_src = d.beta;
    T.X = P.take(sizeof(uint64_t) * (size_t)d.K * (N + 1));
    T.x = P.take(sizeof(double) * (size_t)d.K * (N + 1));
    T.T = P.take(sizeof(uint64_t) * 2 * d.K);
    T.beta = P.take(sizeof(double) * d.K);
}

Layout plan(const pa_run_desc *runs, int n_runs, pa_repr repr)
{
    Layout Lo;
    Planner P;
    Lo.npop_ctx = 1;
    Lo.Kmax = 0;
    Lo.maxN = 0;
    for (int r = 0; r < n_runs; ++r) {
        Lo.npop_ctx = std::max(Lo.npop_ctx, n_pop_of(runs[r].overlap));
        Lo.Kmax = std::max(Lo.Kmax, runs[r].K);
        Lo.maxN = std::max(Lo.maxN, runs[r].L * runs[r].L);
    }
    Lo.runinfo = P.take(sizeof(RunInfo) * n_runs);
    Lo.popstate = P.take(sizeof(PopState) * n_runs * MAX_POP);
    Lo.dseed = P.take(sizeof(uint64_t) * n_runs);
    Lo.stats = P.take(STAT_BYTES);
    Lo.queue = P.take(sizeof(uint32_t) * 4);
    Lo.n_items = 0;
    Lo.n_chunk_items = 0;
    Lo.n_meas_items = 0;
    for (int r = 0; r < n_runs; ++r) {
        const int npop = n_pop_of(runs[r].overlap);
        Lo.n_items += npop * groups_cap_of(runs[r]);
        Lo.n_chunk_items += npop * chunks_cap_of(runs[r]);
        Lo.n_meas_items += npop * n_meas_items_of(runs[r]);
    }
    Lo.items = P.take(sizeof(Item) * Lo.n_items);
    Lo.meas_items = P.take(sizeof(SweepItem) * Lo.n_meas_items);
    // the batched sweep's list: up to MAX_SWEEP_CHUNKS chunks of every item,
    // and one completion flag per item
    const size_t chunks_max = repr == PA_MSC64 ? MAX_SWEEP_CHUNKS : 1;
    Lo.sweep_items = P.take(sizeof(SweepItem) * Lo.n_items * chunks_max);
    Lo.sweep_flags = P.take(sizeof(uint32_t) * (repr == PA_MSC64 ? Lo.n_items : 1));
    Lo.chunk_items = P.take(sizeof(ChunkItem) * Lo.n_chunk_items);
    Lo.obs = P.take(sizeof(pa_obs) * (size_t)Lo.Kmax * n_runs * Lo.npop_ctx);
    Lo.logw = P.take(sizeof(double) * (size_t)Lo.Kmax * n_runs);
    Lo.qw = P.take(sizeof(double) * (size_t)Lo.Kmax * n_runs);
    Lo.wavg = P.take(sizeof(pa_wavg) * (size_t)Lo.Kmax * n_runs);
    Lo.famst = P.take(sizeof(pa_famstat) * (size_t)Lo.Kmax * n_runs);
    {
        size_t wq = 0;
        for (int r = 0; r < n_runs; ++r)
            if (runs[r].qhist) wq += (size_t)runs[r].K * (runs[r].L * runs[r].L + 1);
        Lo.wq = P.take(sizeof(double) * wq);
    }
    Lo.runs.resize(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        const pa_run_desc &d = runs[r];
        const int N = d.L * d.L;
        int t = -1;
        for (size_t k = 0; k < Lo.tables.size(); ++k)
            if (same_table(Lo.tables[k], N, d)) t = (int)k;
        if (t < 0) {
            TableOff T;
            plan_table(P, N, d, T);
            Lo.tables.push_back(T);
            t = (int)Lo.tables.size() - 1;
        }
        plan_run_buffers(P, d, repr, Lo.runs[r]);
        Lo.runs[r].table = t;
    }
    Lo.total = P.off;
    return Lo;
}

void compute_tables(const pa_run_desc &d, int N, std::vector<uint64_t> &X, std::vector<double> &x,
                    std::vector<uint64_t> &T)
{
    // Reweighting factors of step beta_{i-1} -> beta_i for a replica at
    // E_min + 4k (Eq. (tauBoltz)): x = exp(-dbeta 4k), X = floor(x 2^40).
    // Metropolis thresholds at beta_i: T = floor(exp(-beta dE) 2^32), dE = 4, 8.
    X.assign((size_t)d.K * (N + 1), 0);
    x.assign((size_t)d.K * (N + 1), 0.0);
    T.assign((size_t)2 * d.K, 0);
    for (int i = 0; i < d.K; ++i) {
        const double db = i == 0 ? 0.0 : d.beta[i] - d.beta[i - 1];
        for (int k = 0; k <= N; ++k) {
            const double v = std::exp(-(db * (double)(4 * k)));
            x[(size_t)i * (N + 1) + k] = v;
            X[(size_t)i * (N + 1) + k] = (uint64_t)std::floor(std::ldexp(v, 40));
        }
        for (int q = 0; q < 2; ++q) {
            const double p = std::exp(-(d.beta[i] * (double)(4 * (q + 1))));
            T[2 * i + q] = (uint64_t)std::floor(std::ldexp(p, 32));
        }
    }
}

}  // namespace pa

namespace {

using u128 = unsigned __int128;

// Exact density of states of the periodic L x L ferromagnet (the energy
// distribution that the theta = infinity limit samples).  Kaufman's closed
// form for the torus, written as a polynomial in y = exp(-2 beta), has the
// exact integer counts as coefficients (Beale's route):
//   sum_u g_u y^u = (Q_00 + Q_01 + Q_10 + Q_11) / 2,
// u the number of unsatisfied bonds (E = -2N + 2u), Q_ab the product over
// the momenta p = pi (2k + a) / L, q = pi (2l + b) / L, taken once per pair
// {(p, q), (-p, -q)}, of (1 + y^2)^2 - 2y (1 - y^2)(cos p + cos q), and, for
// a momentum equal to its own negative (p, q in {0, pi}), of the square
// roots 1 - 2y - y^2 (p = q = 0), 1 + 2y - y^2 (p = q = pi), 1 + y^2.
// The product is exact modulo primes P = 1 (mod 2L), in which the 2L-th
// roots of unity, and so the cosines (z^j + z^-j) / 2, exist; enough primes
// for 2^N, and the counts are rebuilt by the Chinese remainder theorem.
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t p)
{
    uint64_t r = 1;
    a %= p;
    for (; e; e >>= 1, a = mulmod(a, a, p))
        if (e & 1) r = mulmod(r, a, p);
    return r;
}

// Deterministic Miller-Rabin for n < 2^64 (these twelve bases suffice).
bool is_prime(uint64_t n)
{
    if (n < 2) return false;
    for (uint64_t q : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++r;
    }
    for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int k = 1; k < r && comp; ++k) {
            x = mulmod(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

// The counts g_u mod P, u = 0 .. 2N.
std::vector<uint64_t> dos_mod(int L, uint64_t P)
{
    const int N = L * L, J = 2 * L;
    // a primitive 2L-th root of unity
    std::vector<int> pf;
    for (int q = 2, m = J; m > 1; ++q)
        if (m % q == 0) {
            pf.push_back(q);
            while (m % q == 0) m /= q;
        }
    uint64_t z = 0;
    for (uint64_t a = 2; !z; ++a) {
        const uint64_t c = powmod(a, (P - 1) / J, P);
        bool prim = true;
        for (int q : pf) prim = prim && powmod(c, J / q, P) != 1;
        if (prim) z = c;
    }
    const uint64_t inv2 = (P + 1) / 2;
    std::vector<uint64_t> cs(J);
    for (int j = 0; j < J; ++j)
        cs[j] = mulmod((powmod(z, j, P) + powmod(z, (uint64_t)(J - j) % J, P)) % P, inv2, P);
    const uint64_t two = 2 % P, minus = P - 1, minus2 = P - 2;
    std::vector<uint64_t> total(2 * N + 1, 0), Q;
    std::vector<char> done((size_t)J * J);
    auto mul = [&](const uint64_t *f, int nf) {   // Q *= f (nf coefficients), in place from the top
        const int d = (int)Q.size();
        Q.resize(d + nf - 1, 0);
        for (int i = d + nf - 2; i >= 0; --i) {
            u128 acc = 0;
            for (int t = 0; t < nf; ++t)
                if (i - t >= 0 && i - t < d) acc += (u128)Q[i - t] * f[t] % P;
            Q[i] = (uint64_t)(acc % P);
        }
    };
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            Q.assign(1, 1);
            std::fill(done.begin(), done.end(), 0);
            for (int k = 0; k < L; ++k)
                for (int l = 0; l < L; ++l) {
                    const int jp = (2 * k + a) % J, jq = (2 * l + b) % J;
                    if (done[(size_t)jp * J + jq]) continue;
                    const int np = (J - jp) % J, nq = (J - jq) % J;
                    done[(size_t)jp * J + jq] = done[(size_t)np * J + nq] = 1;
                    if (np == jp && nq == jq) {   // p, q in {0, pi}: the square root
                        const bool p0 = jp == 0, q0 = jq == 0;
                        uint64_t r[3];
                        if (p0 && q0) { r[0] = 1; r[1] = minus2; r[2] = minus; }           // 1 - 2y - y^2
                        else if (!p0 && !q0) { r[0] = 1; r[1] = two; r[2] = minus; }       // 1 + 2y - y^2
                        else { r[0] = 1; r[1] = 0; r[2] = 1; }                             // 1 + y^2
                        mul(r, 3);
                        continue;
                    }
                    const uint64_t sum = (cs[jp] + cs[jq]) % P, s2 = mulmod(two, sum, P);
                    const uint64_t f[5] = {1, (P - s2) % P, two, s2, 1};   // 1 - 2sy + 2y^2 + 2sy^3 + y^4
                    mul(f, 5);
                }
            for (int u = 0; u <= 2 * N; ++u) total[u] = (total[u] + Q[u]) % P;
        }
    for (auto &v : total) v = mulmod(v, inv2, P);
    return total;
}

// Multi-limb unsigned integers, little-endian 64-bit limbs.
using Big = std::vector<uint64_t>;

void big_mul_add(Big &x, uint64_t m, uint64_t a)   // x = x m + a
{
    u128 carry = a;
    for (auto &w : x) {
        const u128 t = (u128)w * m + carry;
        w = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) x.push_back((uint64_t)carry);
}

// g_m for E = -2N + 4m, m = 0 .. N (exact), or empty if a check fails.
std::vector<Big> fm_dos_exact(int L)
{
    const int N = L * L;
    const int nprimes = (N + 2) / 61 + 2;   // product of primes > 2^(61 nprimes) > 2^(N + 2)
    std::vector<uint64_t> primes;
    const uint64_t J = 2 * (uint64_t)L;
    for (uint64_t k = ((1ull << 62) - 1) / J; primes.size() < (size_t)nprimes && k > 0; --k)
        if (is_prime(k * J + 1)) primes.push_back(k * J + 1);
    std::vector<std::vector<uint64_t>> res;
    for (uint64_t P : primes) res.push_back(dos_mod(L, P));
    // Garner: mixed-radix digits v_i, then x = v_0 + p_0 (v_1 + p_1 (v_2 + ...))
    const int k = (int)primes.size();
    std::vector<uint64_t> inv((size_t)k * k, 0);   // inv[i k + j] = p_j^-1 mod p_i
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) inv[(size_t)i * k + j] = powmod(primes[j] % primes[i], primes[i] - 2, primes[i]);
    std::vector<Big> g(N + 1);
    Big sum;
    for (int u = 0; u <= 2 * N; ++u) {
        std::vector<uint64_t> v(k);
        for (int i = 0; i < k; ++i) {
            uint64_t x = res[i][u];
            for (int j = 0; j < i; ++j)
                x = mulmod((x + primes[i] - v[j] % primes[i]) % primes[i], inv[(size_t)i * k + j], primes[i]);
            v[i] = x;
        }
        Big x{v[k - 1]};
        for (int i = k - 2; i >= 0; --i) big_mul_add(x, primes[i], v[i]);
        while (x.size() > 1 && x.back() == 0) x.pop_back();
        if (u & 1) {
            if (x.size() != 1 || x[0] != 0) return {};   // odd u never occurs on the torus
            continue;
        }
        g[u / 2] = x;
        // running sum for the check sum_m g_m = 2^N
        if (sum.size() < x.size()) sum.resize(x.size(), 0);
        u128 carry = 0;
        for (size_t w = 0; w < sum.size(); ++w) {
            const u128 t = (u128)sum[w] + (w < x.size() ? x[w] : 0) + carry;
            sum[w] = (uint64_t)t;
            carry = t >> 64;
        }
        if (carry) sum.push_back((uint64_t)carry);
    }
    Big want((size_t)N / 64 + 1, 0);
    want[N / 64] = 1ull << (N % 64);
    while (sum.size() > 1 && sum.back() == 0) sum.pop_back();
    while (want.size() > 1 && want.back() == 0) want.pop_back();
    if (sum != want) return {};
    return g;
}

// g_m, cached per L (empty if L is outside 4..30, odd, or a check failed).
const std::vector<Big> &fm_dos(int L)
{
    static std::mutex mu;
    static std::map<int, std::vector<Big>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(L);
    if (it == cache.end()) {
        std::vector<Big> g;
        if (L >= 4 && L <= 30 && (L & 1) == 0) g = fm_dos_exact(L);
        it = cache.emplace(L, std::move(g)).first;
    }
    return it->second;
}

// The nearest double to a multi-limb integer (ties to even).
double big_to_double(const Big &x)
{
    int top = (int)x.size() - 1;
    while (top > 0 && x[top] == 0) --top;
    if (top == 0) return (double)x[0];   // one limb: the conversion rounds to nearest
    const int hb = 63 - __builtin_clzll(x[top]);   // highest set bit within the top limb
    const int msb = 64 * top + hb;                  // of the whole number
    // the 64 bits below and including the highest set bit, and a sticky bit
    const int lo = msb - 63;
    auto bit_word = [&](int from) -> uint64_t {      // 64 bits starting at bit `from`
        const int w = from / 64, o = from % 64;
        uint64_t v = x[w] >> o;
        if (o && w + 1 < (int)x.size()) v |= x[w + 1] << (64 - o);
        return v;
    };
    const uint64_t t = bit_word(lo);
    bool sticky = false;
    for (int w = 0; w < lo / 64 && !sticky; ++w) sticky = x[w] != 0;
    if (!sticky && lo % 64) sticky = (x[lo / 64] & ((1ull << (lo % 64)) - 1)) != 0;
    uint64_t mant = t >> 11;   // 53 bits
    const uint64_t rem = t & 0x7FF, half = 0x400;
    if (rem > half || (rem == half && (sticky || (mant & 1)))) ++mant;
    return std::ldexp((double)mant, lo + 11);
}

}  // namespace

namespace pa {

bool dos_thresholds(const pa_run_desc &d, std::vector<uint64_t> &out)
{
    const std::vector<Big> &g = fm_dos(d.L);
    if (g.empty()) return false;
    const int N = d.L * d.L;
    std::vector<double> gd(N + 1);
    for (int m = 0; m <= N; ++m) gd[m] = big_to_double(g[m]);
    out.assign((size_t)d.K * (N + 1), 0);
    std::vector<double> S(N + 1);
    for (int i = 0; i < d.K; ++i) {
        double acc = 0.0;
        for (int m = 0; m <= N; ++m) {
            acc += gd[m] * std::exp(-4.0 * d.beta[i] * (double)m);
            S[m] = acc;
        }
        for (int m = 0; m <= N; ++m) {
            const double q = S[m] / acc;
            out[(size_t)i * (N + 1) + m] = q >= 1.0 ? UINT64_MAX : (uint64_t)std::ldexp(q, 64);
        }
    }
    return true;
}

RunInfo make_runinfo(const pa_run_desc &d, uint8_t *base, const RunOff &o, uint8_t *tbase, const TableOff &T,
                     pa_obs *obs, int obs_stride, int obs_off)
{
    RunInfo I;
    std::memset(&I, 0, sizeof(I));
    I.L = d.L;
    I.N = d.L * d.L;
    I.npop = n_pop_of(d.overlap);
    I.R = d.R;
    I.R_cap = d.R_cap;
    I.theta = d.theta == PA_THETA_EXACT ? 0 : d.theta;   // no Metropolis sweeps at theta = infinity
    I.exact_dos = d.theta == PA_THETA_EXACT ? 1 : 0;
    I.K = d.K;
    I.model = d.model;
    I.resampling = d.resampling;
    I.overlap = d.overlap;
    I.qhist = d.qhist;
    I.groups_cap = groups_cap_of(d);
    I.key0 = (uint32_t)(d.seed & 0xffffffffu);
    I.key1 = (uint32_t)(d.seed >> 32);
    I.obs_stride = obs_stride;
    I.obs_off = obs_off;
    for (int p = 0; p < I.npop; ++p) {
        for (int b = 0; b < 2; ++b) {
            I.spins[p][b] = base + o.spins[p][b];
            I.E[p][b] = (int32_t *)(base + o.E[p][b]);
            I.fam[p][b] = (int32_t *)(base + o.fam[p][b]);
        }
        I.r[p] = (int32_t *)(base + o.r[p]);
        I.C[p] = (int32_t *)(base + o.C[p]);
        I.parent[p] = (int32_t *)(base + o.parent[p]);
        I.P[p] = d.resampling == PA_MULTINOMIAL ? (uint64_t *)(base + o.P[p]) : nullptr;
        I.part[p] = (int64_t *)(base + o.part[p]);
        I.partS[p] = (double *)(base + o.partS[p]);
        I.tot64[p] = (uint64_t *)(base + o.tot64[p]);
        I.base64[p] = (uint64_t *)(base + o.base64[p]);
        I.tot32[p] = (int32_t *)(base + o.tot32[p]);
        I.base32[p] = (int32_t *)(base + o.base32[p]);
    }
    I.obs = obs;
    I.qh = d.qhist ? (int32_t *)(base + o.qh) : nullptr;
    I.jbits = base + o.jbits;
    I.wang = is_wang(d.overlap) ? (int32_t *)(base + o.wang) : nullptr;
    I.wang_lb = wang_lb_of(d.R_cap);
    I.tabD = d.theta == PA_THETA_EXACT ? (const uint64_t *)(base + o.dos) : nullptr;
    I.tabX = (const uint64_t *)(tbase + T.X);
    I.tabx = (const double *)(tbase + T.x);
    I.tabT = (const uint64_t *)(tbase + T.T);
    I.beta = (const double *)(tbase + T.beta);
    return I;
}

PopState initial_popstate(const pa_run_desc &d)
{
    PopState S;
    std::memset(&S, 0, sizeof(S));
    S.i = 0;
    S.cur = 0;
    S.src = 0;
    S.Rprev = d.R;
    S.Rcur = d.R;
    S.status = PA_OK;
    S.moved = 1;
    S.A = (double)d.L * d.L * std::log(2.0);   // ln Z(0) = N ln 2
    S.EminAcc = INT32_MAX;
    return S;
}

void meas_items_of(const pa_run_desc &d, int run, int pop, std::vector<SweepItem> &out)
{
    const int gpw = MEAS_WAVES / meas_waves_per_group(d.L * d.L);
    for (int g = 0; g < groups_cap_of(d); g += gpw) out.push_back({run, pop, g, std::min(gpw, groups_cap_of(d) - g)});
}

int wang_lds_ints_of(const pa_run_desc *const *runs, int n, int lds_limit)
{
    int best = 0;
    for (int r = 0; r < n; ++r)
        if (is_wang(runs[r]->overlap) && 8 * (size_t)runs[r]->R_cap + 256 <= (size_t)lds_limit)
            best = std::max(best, runs[r]->R_cap);
    return 2 * best;
}

int default_groups(int L)
{
    const int nh = L * L / 2;
    int G = (2048 + nh / 2) / nh;
    return G < 1 ? 1 : (G > 64 ? 64 : G);
}

pa_status dev_fail(pa_ctx *c, hipError_t e)
{
    c->failed = true;
    if (e == hipSuccess) e = hipGetLastError();
    if (c->last == hipSuccess) c->last = e;
    return PA_ERR_DEVICE;
}

int groups_for(const pa_ctx *c, int L)
{
    auto it = c->groups_per_wg.find(L);
    return it == c->groups_per_wg.end() ? default_groups(L) : it->second;
}

// Work list and LDS size of the batched sweep for the current tuning.
// Returns false if some lattice block does not fit in LDS.
bool plan_sweep(const pa_ctx *c, std::vector<SweepItem> &items, size_t &lds)
{
    items.clear();
    lds = 0;
    for (int r = 0; r < c->n_runs; ++r) {
        const pa_run_desc &d = c->descs[r];
        const int N = d.L * d.L;
        if ((size_t)groups_for(c, d.L) * N > 65535) return false;   // 16-bit LDS word indices
        // the larger, whole-list size: the kernel the plan launches is chosen later
        lds = std::max(lds, msc_lds_bytes(N, groups_for(c, d.L), d.model == PA_EA_PMJ, c->sweep_threads,
                                          c->sweep_dense | (c->sweep_pooled ? 1 << 8 : 0) | MSC_WHOLE_LISTS));
    }
    if (lds > (size_t)c->lds_limit) return false;
    for (int r = 0; r < c->n_runs; ++r) {
        const pa_run_desc &d = c->descs[r];
        const int G = groups_for(c, d.L);
        for (int p = 0; p < n_pop_of(d.overlap); ++p)
            for (int g = 0; g < groups_cap_of(d); g += G)
                items.push_back({r, p, g, std::min(G, groups_cap_of(d) - g)});
    }
    // largest items first (words of lattice per item), so the cheapest ones
    // fill the tail of the launch; ties keep run order
    std::stable_sort(items.begin(), items.end(), [c](const SweepItem &a, const SweepItem &b) {
        const long wa = (long)a.ngroups * c->descs[a.run].L * c->descs[a.run].L;
        const long wb = (long)b.ngroups * c->descs[b.run].L * c->descs[b.run].L;
        return wa > wb;
    });
    return true;
}

pa_status upload_sweep_plan(pa_ctx *c)
{
    std::vector<SweepItem> items;
    size_t lds = 0;
    if (!plan_sweep(c, items, lds)) return PA_ERR_ARG;
    std::vector<int> run_L(c->n_runs), run_ea(c->n_runs);
    for (int r = 0; r < c->n_runs; ++r) {
        run_L[r] = c->descs[r].theta > 0 ? c->descs[r].L : 0;
        run_ea[r] = c->descs[r].model == PA_EA_PMJ;
    }
    SweepClass cls[MAX_SWEEP_CLASSES];
    if (prepare_msc_lds(lds) != hipSuccess) return dev_fail(c);
    const int ncls = sweep_classes(items, run_L, run_ea, cls, c->sweep_threads,
                                   c->sweep_dense | (c->sweep_pooled ? 1 << 8 : 0), true);
    if (ncls < 0) return PA_ERR_ARG;
    if (!sweep_class_grids(cls, ncls, c->sweep_threads, c->sweep_persistent)) return dev_fail(c);
    if (ncls == 1 && cls[0].grid > 0 && cls[0].grid < cls[0].count) {
        const int K = c->sweep_chunks > 0 ? c->sweep_chunks : sweep_chunks_auto(cls[0].count, cls[0].grid);
        std::vector<int> run_theta(c->n_runs);
        for (int r = 0; r < c->n_runs; ++r) run_theta[r] = std::max(0, c->descs[r].theta);
        if (expand_sweep_chunks(items, cls[0], K, run_theta) != 0) return PA_ERR_ARG;
    }
    if (!items.empty())
        PA_HIP(c, hipMemcpyAsync(at<SweepItem>(c, c->lo.sweep_items), items.data(),
                                 sizeof(SweepItem) * items.size(), hipMemcpyHostToDevice, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    c->lc.sweep_items = at<SweepItem>(c, c->lo.sweep_items);
    c->lc.sweep_flags = at<unsigned int>(c, c->lo.sweep_flags);
    c->lc.n_sweep_items = (int)items.size();
    c->lc.sweep_threads = c->sweep_threads;
    c->lc.sweep_dense = c->sweep_dense;
    c->lc.sweep_pooled = c->sweep_pooled ? 1 : 0;
    c->lc.n_sweep_classes = ncls;
    std::copy(cls, cls + ncls, c->lc.sweep_cls);
    return PA_OK;
}

pa_status enqueue_step(pa_ctx *c)
{
    if (launch_anneal(c->lc) != hipSuccess) return dev_fail(c);
    if (launch_resample(c->lc) != hipSuccess) return dev_fail(c);
    if (c->repr == PA_MSC64) {
        if (launch_sweep_msc(c->lc) != hipSuccess) return dev_fail(c);
    } else {
        for (int r = 0; r < c->n_runs; ++r) {
            const pa_run_desc &d = c->descs[r];
            if (launch_sweep_int8_run(c->lc, r, d.L, groups_cap_of(d), n_pop_of(d.overlap), d.theta) !=
                hipSuccess)
                return dev_fail(c);
        }
    }
    if (launch_dos_sample(c->lc) != hipSuccess) return dev_fail(c);
    if (launch_measure(c->lc) != hipSuccess) return dev_fail(c);
    return PA_OK;
}

pa_status read_stats(pa_ctx *c, uint64_t out[3])
{
    std::vector<uint64_t> slots((size_t)NSTAT * STAT_SLOTS);
    PA_HIP(c, hipMemcpyAsync(slots.data(), c->lc.stats, STAT_BYTES, hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < 3; ++k) {
        out[k] = 0;
        for (int q = 0; q < STAT_SLOTS; ++q) out[k] += slots[(size_t)q * NSTAT + k];
    }
    uint64_t stalls = 0;
    for (int q = 0; q < STAT_SLOTS; ++q) stalls += slots[(size_t)q * NSTAT + ST_STALL];
    return stalls ? PA_ERR_STATE : PA_OK;
}

// A captured step graph holds the launch shapes it was captured with.
void drop_graph(pa_ctx *c)
{
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    if (c->graph_def) {
        (void)hipGraphDestroy(c->graph_def);
        c->graph_def = nullptr;
    }
}

}  // namespace pa

extern "C" {

const char *pa_status_str(pa_status st)
{
    switch (st) {
    case PA_OK: return "ok";
    case PA_ERR_ARG: return "invalid argument";
    case PA_ERR_NOMEM: return "workspace too small";
    case PA_ERR_CAPACITY: return "population exceeded its capacity";
    case PA_ERR_STATE: return "call out of order";
    case PA_ERR_NUMERIC: return "numeric failure (empty population or non-finite value)";
    case PA_ERR_DEVICE: return "HIP device error";
    }
    return "unknown status";
}

pa_status pa_workspace_size(const pa_run_desc *runs, int32_t n_runs, pa_repr repr, size_t *bytes)
{
    if (!runs || n_runs < 1 || !bytes || (repr != PA_INT8 && repr != PA_MSC64)) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r)
        if (!desc_ok(runs[r], repr)) return PA_ERR_ARG;
    *bytes = plan(runs, n_runs, repr).total;
    return PA_OK;
}

pa_status pa_create(const pa_run_desc *runs, int32_t n_runs, pa_repr repr, void *dev_workspace, size_t bytes,
                    void *hip_stream, pa_ctx **out)
{
    if (!out) return PA_ERR_ARG;
    *out = nullptr;
    size_t need = 0;
    pa_status st = pa_workspace_size(runs, n_runs, repr, &need);
    if (st != PA_OK) return st;
    if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return PA_ERR_ARG;
    if (bytes < need) return PA_ERR_NOMEM;

    pa_ctx *c = new pa_ctx();
    c->n_runs = n_runs;
    c->repr = repr;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (uint8_t *)dev_workspace;
    c->lo = plan(runs, n_runs, repr);
    c->descs.assign(runs, runs + n_runs);
    c->betas.resize(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        c->betas[r].assign(runs[r].beta, runs[r].beta + runs[r].K);
        c->descs[r].beta = c->betas[r].data();
        if (runs[r].resampling == PA_MULTINOMIAL) c->any_multinomial = true;
        if (is_wang(runs[r].overlap)) c->any_wang = true;
        if (runs[r].theta == PA_THETA_EXACT) c->any_exact_dos = true;
    }
    // table sources must point at the context's own copies
    for (auto &t : c->lo.tables) {
        for (int r = 0; r < n_runs; ++r)
            if (t.beta_src == runs[r].beta) {
                t.beta_src = c->betas[r].data();
                break;
            }
    }
    const Layout &Lo = c->lo;

    // host images of the device-side records
    c->hinfo.resize(n_runs);
    std::vector<PopState> hst((size_t)n_runs * MAX_POP);
    std::vector<Item> items;
    std::vector<ChunkItem> chunks;
    std::vector<SweepItem> meas;
    std::vector<uint64_t> dseed(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        const pa_run_desc &d = c->descs[r];
        const RunOff &o = Lo.runs[r];
        const TableOff &T = Lo.tables[o.table];
        c->hinfo[r] = make_runinfo(d, c->ws, o, c->ws, T, at<pa_obs>(c, Lo.obs), n_runs * Lo.npop_ctx,
                                   r * Lo.npop_ctx);
        for (int p = 0; p < n_pop_of(d.overlap); ++p) {
            hst[(size_t)r * MAX_POP + p] = initial_popstate(d);
            for (int g = 0; g < groups_cap_of(d); ++g) items.push_back({r, p, g, 0});
            for (int k = 0; k < chunks_cap_of(d); ++k) chunks.push_back({r, p, k, 0});
            meas_items_of(d, r, p, meas);
        }
        dseed[r] = d.disorder_seed;
    }

    c->lc.runs = at<RunInfo>(c, Lo.runinfo);
    c->lc.st = at<PopState>(c, Lo.popstate);
    c->lc.items = at<Item>(c, Lo.items);
    c->lc.n_items = Lo.n_items;
    c->lc.chunk_items = at<ChunkItem>(c, Lo.chunk_items);
    c->lc.n_chunk_items = Lo.n_chunk_items;
    c->lc.meas_items = at<SweepItem>(c, Lo.meas_items);
    c->lc.n_meas_items = Lo.n_meas_items;
    c->lc.run0 = 0;
    c->lc.n_runs = n_runs;
    c->lc.npop_ctx = Lo.npop_ctx;
    c->lc.repr = repr;
    c->lc.any_multinomial = c->any_multinomial;
    c->lc.mn_split = 1;
    c->lc.any_overlap = false;
    // copy workgroups per item: each wavefront keeps about four 64-site blocks
    // of its group (L = 64: 40 -> 35 us per copy at R = 1e5 against one
    // workgroup per item); set by the smallest lattice of the context
    int min_n = 1 << 30;
    for (int r = 0; r < n_runs; ++r) min_n = std::min(min_n, runs[r].L * runs[r].L);
    {
        const int blocks_per_wave = (min_n / 64) / meas_waves_per_group(min_n);
        c->lc.copy_split = std::max(1, std::min(4, blocks_per_wave / 4));
    }
    for (int r = 0; r < n_runs; ++r) {
        if (runs[r].resampling == PA_MULTINOMIAL && runs[r].R > CH) c->lc.mn_split = CH_PER;
        if (runs[r].overlap != PA_Q_NONE) c->lc.any_overlap = true;
    }
    c->lc.any_wang = c->any_wang;
    c->lc.any_exact_dos = c->any_exact_dos;
    c->lc.stats = at<unsigned long long>(c, Lo.stats);
    c->lc.sweep_queue = at<unsigned int>(c, Lo.queue);
    c->lc.n_sweep_classes = 0;
    c->lc.stream = c->stream;

    auto fail = [&](pa_status s) {
        delete c;
        return s;
    };
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return fail(PA_ERR_DEVICE);
    }
    if (repr == PA_MSC64) {
        std::vector<SweepItem> probe;
        size_t lds = 0;
        if (!plan_sweep(c, probe, lds)) return fail(PA_ERR_ARG);
    }
    if (c->any_wang) {
        std::vector<const pa_run_desc *> dp(n_runs);
        for (int r = 0; r < n_runs; ++r) dp[r] = &c->descs[r];
        c->lc.wang_lds_ints = wang_lds_ints_of(dp.data(), n_runs, c->lds_limit);
        if (prepare_wang_lds(sizeof(int32_t) * (size_t)c->lc.wang_lds_ints) != hipSuccess) return fail(PA_ERR_DEVICE);
    }

    hipStream_t s = c->stream;
    bool ok = true;
    // one clear of the whole workspace first: the histograms, records,
    // descendant counts and counters that kernels accumulate into start at
    // zero (a single launch, whatever the number of runs)
    ok = ok && launch_fill_u32(c->ws, 0, Lo.total / 4, s) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)c->lc.runs, c->hinfo.data(), sizeof(RunInfo) * n_runs, hipMemcpyHostToDevice, s) ==
                   hipSuccess;
    ok = ok && hipMemcpyAsync(c->lc.st, hst.data(), sizeof(PopState) * hst.size(), hipMemcpyHostToDevice, s) ==
                   hipSuccess;
    ok = ok && hipMemcpyAsync(at<Item>(c, Lo.items), items.data(), sizeof(Item) * items.size(),
                              hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(at<ChunkItem>(c, Lo.chunk_items), chunks.data(), sizeof(ChunkItem) * chunks.size(),
                              hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(at<SweepItem>(c, Lo.meas_items), meas.data(), sizeof(SweepItem) * meas.size(),
                              hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(at<uint64_t>(c, Lo.dseed), dseed.data(), sizeof(uint64_t) * n_runs,
                              hipMemcpyHostToDevice, s) == hipSuccess;
    std::vector<std::vector<uint64_t>> hX(Lo.tables.size()), hT(Lo.tables.size()), hD;
    hD.reserve(n_runs);
    std::vector<std::vector<double>> hx(Lo.tables.size());
    for (size_t t = 0; t < Lo.tables.size() && ok; ++t) {
        const TableOff &T = Lo.tables[t];
        pa_run_desc d = {};
        d.K = T.K;
        d.beta = T.beta_src;
        compute_tables(d, T.N, hX[t], hx[t], hT[t]);
        ok = ok && hipMemcpyAsync(at<uint64_t>(c, T.X), hX[t].data(), sizeof(uint64_t) * hX[t].size(),
                                  hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(at<double>(c, T.x), hx[t].data(), sizeof(double) * hx[t].size(),
                                  hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(at<uint64_t>(c, T.T), hT[t].data(), sizeof(uint64_t) * hT[t].size(),
                                  hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(at<double>(c, T.beta), T.beta_src, sizeof(double) * T.K, hipMemcpyHostToDevice,
                                  s) == hipSuccess;
    }
    for (int r = 0; r < n_runs && ok; ++r) {
        const pa_run_desc &d = c->descs[r];
        const RunOff &o = Lo.runs[r];
        if (d.theta == PA_THETA_EXACT) {   // energy draw thresholds (host copy kept until the sync)
            hD.emplace_back();
            ok = dos_thresholds(d, hD.back()) &&
                 hipMemcpyAsync(at<uint64_t>(c, o.dos), hD.back().data(), sizeof(uint64_t) * hD.back().size(),
                                hipMemcpyHostToDevice, s) == hipSuccess;
        }
    }
    ok = ok && (repr != PA_MSC64 || upload_sweep_plan(c) == PA_OK);
    ok = ok && launch_init(c->lc, at<uint64_t>(c, Lo.dseed)) == hipSuccess;
    ok = ok && launch_measure(c->lc) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) return fail(PA_ERR_DEVICE);
    c->i = 0;
    c->phase = PH_MEASURED;
    *out = c;
    return PA_OK;
}

pa_status pa_anneal_step(pa_ctx *c, int32_t i)
{
    if (!c) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED || i != c->i + 1 || i >= c->lo.Kmax) return PA_ERR_STATE;
    if (launch_anneal(c->lc) != hipSuccess) return dev_fail(c);
    c->i = i;
    c->phase = PH_ANNEALED;
    return PA_OK;
}

pa_status pa_resample(pa_ctx *c, int32_t i)
{
    if (!c) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_ANNEALED || i != c->i) return PA_ERR_STATE;
    if (launch_resample(c->lc) != hipSuccess) return dev_fail(c);
    c->phase = PH_RESAMPLED;
    return PA_OK;
}

pa_status pa_sweep(pa_ctx *c, int32_t i)
{
    if (!c) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_RESAMPLED || i != c->i) return PA_ERR_STATE;
    if (c->repr == PA_MSC64) {
        if (launch_sweep_msc(c->lc) != hipSuccess) return dev_fail(c);
    } else {
        for (int r = 0; r < c->n_runs; ++r) {
            const pa_run_desc &d = c->descs[r];
            if (launch_sweep_int8_run(c->lc, r, d.L, groups_cap_of(d), n_pop_of(d.overlap), d.theta) != hipSuccess)
                return dev_fail(c);
        }
    }
    if (launch_dos_sample(c->lc) != hipSuccess) return dev_fail(c);
    c->phase = PH_SWEPT;
    return PA_OK;
}

pa_status pa_measure(pa_ctx *c, int32_t i, pa_obs *host_out)
{
    if (!c) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_SWEPT || i != c->i) return PA_ERR_STATE;
    if (launch_measure(c->lc) != hipSuccess) return dev_fail(c);
    c->phase = PH_MEASURED;
    if (host_out) {
        const size_t n = (size_t)c->n_runs * c->lo.npop_ctx;
        PA_HIP(c, hipMemcpyAsync(host_out, at<pa_obs>(c, c->lo.obs) + (size_t)i * n, sizeof(pa_obs) * n,
                                 hipMemcpyDeviceToHost, c->stream));
        PA_HIP(c, hipStreamSynchronize(c->stream));
    }
    return PA_OK;
}

pa_status pa_run(pa_ctx *c, int32_t i_begin, int32_t i_end)
{
    if (!c) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED || i_begin != c->i + 1 || i_end > c->lo.Kmax || i_end <= i_begin)
        return PA_ERR_STATE;
    if (!c->graph) {
        // One temperature step: every kernel reads its temperature index and
        // buffers from device state, so the same graph serves every step.
        // Capture runs on a private stream (the caller's may be the null
        // stream, which cannot be captured); replays go to the caller's.
        if (!c->cap_stream) PA_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        c->lc.stream = c->cap_stream;
        const hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (eb != hipSuccess) {
            c->lc.stream = c->stream;
            return dev_fail(c, eb);
        }
        pa_status st = enqueue_step(c);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        c->lc.stream = c->stream;
        if (st != PA_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return dev_fail(c, e);
        }
        c->graph_def = g;
        PA_HIP(c, hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0));
    }
    for (int i = i_begin; i < i_end; ++i) PA_HIP(c, hipGraphLaunch(c->graph, c->stream));
    c->i = i_end - 1;
    c->phase = PH_MEASURED;
    return PA_OK;
}

namespace {

// Groups of M runs with one L and schedule each, population pop present.
bool groups_ok(const pa_ctx *c, int M, int pop, bool need_qhist)
{
    if (M < 1 || c->n_runs % M != 0) return false;
    const int K = c->descs[0].K;
    for (int r = 0; r < c->n_runs; ++r) {
        const pa_run_desc &d = c->descs[r];
        if (d.K != K || pop < 0 || pop >= n_pop_of(d.overlap)) return false;
        if (need_qhist && !d.qhist) return false;
        const pa_run_desc &d0 = c->descs[(r / M) * M];
        if (d.L != d0.L || std::memcmp(d.beta, d0.beta, sizeof(double) * K) != 0) return false;
    }
    return true;
}

bool kind_ok(int kind) { return kind >= 0 && kind <= (PA_W_SIMPLE | PA_W_EXCLUDE_LARGE_FAMILY); }

}  // namespace

pa_status pa_weighted_average(pa_ctx *c, int32_t M, int32_t kind, int32_t pop, pa_wavg *host_out)
{
    if (!c || !host_out || !kind_ok(kind) || !groups_ok(c, M, pop, false)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const int K = c->descs[0].K;
    const int i_done = c->phase == PH_MEASURED ? c->i : c->i - 1;
    pa_wavg *dout = at<pa_wavg>(c, c->lo.wavg);
    if (launch_wavg(c->lc, at<pa_obs>(c, c->lo.obs), M, kind, pop, K, i_done, at<double>(c, c->lo.logw),
                    at<double>(c, c->lo.qw), dout) != hipSuccess)
        return dev_fail(c);
    PA_HIP(c, hipMemcpyAsync(host_out, dout, sizeof(pa_wavg) * (size_t)(c->n_runs / M) * K, hipMemcpyDeviceToHost,
                             c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    return PA_OK;
}

pa_status pa_weighted_qhist(pa_ctx *c, int32_t M, int32_t kind, int32_t pop, double *host_out)
{
    if (!c || !host_out || !kind_ok(kind) || !groups_ok(c, M, pop, true)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const int K = c->descs[0].K;
    const int N = c->descs[0].L * c->descs[0].L;   // every group must have it (checked above per group)
    for (int r = 0; r < c->n_runs; ++r)
        if (c->descs[r].L * c->descs[r].L != N) return PA_ERR_ARG;   // one bin count for the output array
    const int i_done = c->phase == PH_MEASURED ? c->i : c->i - 1;
    double *dout = at<double>(c, c->lo.wq);
    if (launch_wqhist(c->lc, at<pa_obs>(c, c->lo.obs), M, kind, pop, K, i_done, at<double>(c, c->lo.logw),
                      at<double>(c, c->lo.qw), dout) != hipSuccess)
        return dev_fail(c);
    const size_t n = (size_t)(c->n_runs / M) * K * (N + 1);
    PA_HIP(c, hipMemcpyAsync(host_out, dout, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    return PA_OK;
}

pa_status pa_family_stats(pa_ctx *c, int32_t pop, pa_famstat *host_out)
{
    if (!c || !host_out || pop < 0 || pop >= c->lo.npop_ctx) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const int K = c->lo.Kmax;
    const int i_done = c->phase == PH_MEASURED ? c->i : c->i - 1;
    pa_famstat *dout = at<pa_famstat>(c, c->lo.famst);
    if (launch_famstats(c->lc, at<pa_obs>(c, c->lo.obs), pop, K, i_done, dout) != hipSuccess) return dev_fail(c);
    PA_HIP(c, hipMemcpyAsync(host_out, dout, sizeof(pa_famstat) * (size_t)c->n_runs * K, hipMemcpyDeviceToHost,
                             c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    return PA_OK;
}

pa_status pa_read_obs(pa_ctx *c, pa_obs *host_out)
{
    if (!c || !host_out) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const int np = c->lo.npop_ctx, K = c->lo.Kmax;
    std::vector<pa_obs> tmp((size_t)K * c->n_runs * np);
    PA_HIP(c, hipMemcpyAsync(tmp.data(), at<pa_obs>(c, c->lo.obs), sizeof(pa_obs) * tmp.size(),
                             hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    for (int r = 0; r < c->n_runs; ++r)
        for (int p = 0; p < np; ++p)
            for (int i = 0; i < K; ++i)
                host_out[((size_t)r * np + p) * K + i] = tmp[((size_t)i * c->n_runs + r) * np + p];
    return PA_OK;
}

pa_status pa_read_qhist(pa_ctx *c, int32_t run, int32_t *host_out)
{
    if (!c || !host_out || run < 0 || run >= c->n_runs || !c->descs[run].qhist) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const pa_run_desc &d = c->descs[run];
    const size_t n = (size_t)n_pop_of(d.overlap) * d.K * (d.L * d.L + 1);
    PA_HIP(c, hipMemcpyAsync(host_out, at<int32_t>(c, c->lo.runs[run].qh), sizeof(int32_t) * n,
                             hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    return PA_OK;
}

pa_status pa_calibrate_philox(void *hip_stream, int32_t calls_per_chain, double *calls_per_s)
{
    if (calls_per_chain < 1 || calls_per_chain > (1 << 20) || !calls_per_s) return PA_ERR_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int blocks = 0, threads = 0;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    ok = ok && launch_philox_rate(1, s, &blocks, &threads) == hipSuccess;   // warm-up
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    ok = ok && launch_philox_rate(calls_per_chain, s, &blocks, &threads) == hipSuccess;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!ok) return PA_ERR_DEVICE;
    *calls_per_s = 2.0 * calls_per_chain * (double)blocks * threads / (ms * 1e-3);
    return PA_OK;
}

pa_status pa_exact_dos_wide(int32_t L, int32_t limbs, uint64_t *host_out)
{
    if (L < 4 || L > 30 || (L & 1) || !host_out || limbs < L * L / 64 + 1) return PA_ERR_ARG;
    const std::vector<Big> &g = fm_dos(L);
    if (g.empty()) return PA_ERR_NUMERIC;
    for (int m = 0; m <= L * L; ++m)
        for (int w = 0; w < limbs; ++w) host_out[(size_t)m * limbs + w] = w < (int)g[m].size() ? g[m][w] : 0;
    return PA_OK;
}

pa_status pa_exact_dos(int32_t L, uint64_t *host_out)
{
    if (L < 4 || L > 10 || (L & 1) || !host_out) return PA_ERR_ARG;
    return pa_exact_dos_wide(L, 2, host_out);
}

pa_status pa_read_pairing(pa_ctx *c, int32_t run, int32_t *host_pairs, int32_t *status, int32_t *R_i)
{
    if (!c || run < 0 || run >= c->n_runs || !host_pairs) return PA_ERR_ARG;
    const pa_run_desc &d = c->descs[run];
    if (!is_wang(d.overlap)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED) return PA_ERR_STATE;
    PopState S;
    PA_HIP(c, hipMemcpyAsync(&S, c->lc.st + (size_t)run * MAX_POP, sizeof(S), hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    const RunInfo &I = c->hinfo[run];
    const WangBufs W = wang_bufs(I.wang, I.R_cap, I.wang_lb);
    int32_t hdr[4];
    PA_HIP(c, hipMemcpyAsync(hdr, W.hdr, sizeof(hdr), hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipMemcpyAsync(host_pairs, W.pi, sizeof(int32_t) * S.Rcur, hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    if (status) *status = hdr[0];
    if (R_i) *R_i = S.Rcur;
    return PA_OK;
}

pa_status pa_read_state(pa_ctx *c, int32_t run, int32_t pop, int8_t *spins, int32_t *E, int32_t *fam,
                        int32_t *counts, int32_t *R_i, int32_t *R_prev)
{
    if (!c || run < 0 || run >= c->n_runs) return PA_ERR_ARG;
    const pa_run_desc &d = c->descs[run];
    if (pop < 0 || pop >= n_pop_of(d.overlap)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    PopState S;
    PA_HIP(c, hipMemcpyAsync(&S, c->lc.st + (size_t)run * MAX_POP + pop, sizeof(S), hipMemcpyDeviceToHost,
                             c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    const RunOff &o = c->lo.runs[run];
    const int N = d.L * d.L;
    const int cur = S.cur;
    if (spins) {
        const size_t site_bytes = c->repr == PA_MSC64 ? 8 : 64;
        std::vector<uint8_t> raw((size_t)groups_cap_of(d) * N * site_bytes);
        PA_HIP(c, hipMemcpyAsync(raw.data(), at<uint8_t>(c, o.spins[pop][cur]), raw.size(), hipMemcpyDeviceToHost,
                                 c->stream));
        PA_HIP(c, hipStreamSynchronize(c->stream));
        for (int j = 0; j < S.Rcur; ++j) {
            const int g = j >> 6, b = j & 63;
            for (int n = 0; n < N; ++n) {
                int down;
                if (c->repr == PA_MSC64) {
                    uint64_t w;
                    std::memcpy(&w, &raw[((size_t)g * N + n) * 8], 8);
                    down = (int)((w >> b) & 1u);
                } else {
                    down = raw[((size_t)g * N + n) * 64 + b] >> 7;
                }
                spins[(size_t)j * N + n] = down ? -1 : 1;
            }
        }
    }
    if (E)
        PA_HIP(c, hipMemcpyAsync(E, at<int32_t>(c, o.E[pop][cur]), sizeof(int32_t) * S.Rcur, hipMemcpyDeviceToHost,
                                 c->stream));
    if (fam)
        PA_HIP(c, hipMemcpyAsync(fam, at<int32_t>(c, o.fam[pop][cur]), sizeof(int32_t) * S.Rcur,
                                 hipMemcpyDeviceToHost, c->stream));
    if (counts)
        PA_HIP(c, hipMemcpyAsync(counts, at<int32_t>(c, o.r[pop]), sizeof(int32_t) * S.Rprev,
                                 hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    if (R_i) *R_i = S.Rcur;
    if (R_prev) *R_prev = S.Rprev;
    return PA_OK;
}

pa_status pa_checkpoint(pa_ctx *c, void *host_buf, size_t *bytes)
{
    if (!c || !bytes) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    const size_t need = sizeof(CkptHeader) + c->lo.total;
    if (!host_buf) {
        *bytes = need;
        return PA_OK;
    }
    if (*bytes < need) return PA_ERR_ARG;
    CkptHeader h = {CKPT_MAGIC, CKPT_VERSION, (uint32_t)c->repr, c->lo.total, c->n_runs, c->i, c->phase,
                    c->lo.npop_ctx, descs_hash(c)};
    std::memcpy(host_buf, &h, sizeof(h));
    PA_HIP(c, hipMemcpyAsync((uint8_t *)host_buf + sizeof(h), c->ws, c->lo.total, hipMemcpyDeviceToHost, c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return PA_OK;
}

pa_status pa_restore(pa_ctx *c, const void *host_buf, size_t bytes)
{
    if (!c || !host_buf || bytes < sizeof(CkptHeader)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (h.magic != CKPT_MAGIC || h.version != CKPT_VERSION || h.repr != (uint32_t)c->repr ||
        h.ws_used != c->lo.total || h.n_runs != c->n_runs || h.desc_hash != descs_hash(c) ||
        bytes < sizeof(h) + h.ws_used)
        return PA_ERR_ARG;
    PA_HIP(c, hipMemcpyAsync(c->ws, (const uint8_t *)host_buf + sizeof(h), c->lo.total, hipMemcpyHostToDevice,
                             c->stream));
    // device records hold absolute pointers: rewrite them for this workspace
    PA_HIP(c, hipMemcpyAsync((void *)c->lc.runs, c->hinfo.data(), sizeof(RunInfo) * c->n_runs, hipMemcpyHostToDevice,
                             c->stream));
    PA_HIP(c, hipStreamSynchronize(c->stream));
    c->i = h.i;
    c->phase = h.phase;
    // the workspace copy brought back the sweep list of the plan at
    // checkpoint time; the launches use the current plan, so its list is
    // written again (the tuning may have changed since)
    if (c->repr == PA_MSC64) return upload_sweep_plan(c);
    return PA_OK;
}

pa_status pa_set_tuning(pa_ctx *c, int32_t L, int32_t threads, int32_t groups_per_wg, int32_t dense_calls)
{
    if (!c || L < 4 || (L & 1) || groups_per_wg < 1 || groups_per_wg > 256 || dense_calls < 0 ||
        dense_calls > 16 || (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024))
        return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED) return PA_ERR_STATE;
    const int old_threads = c->sweep_threads, old_dense = c->sweep_dense;
    const auto old_groups = c->groups_per_wg;
    c->sweep_threads = threads;
    c->sweep_dense = dense_calls;
    c->groups_per_wg[L] = groups_per_wg;
    if (c->repr != PA_MSC64) return PA_OK;
    std::vector<SweepItem> probe;
    size_t lds = 0;
    if (!plan_sweep(c, probe, lds)) {
        c->sweep_threads = old_threads;
        c->sweep_dense = old_dense;
        c->groups_per_wg = old_groups;
        return PA_ERR_ARG;
    }
    drop_graph(c);
    return upload_sweep_plan(c);
}

pa_status pa_set_persistent(pa_ctx *c, int32_t on)
{
    if (!c || (on != 0 && on != 1)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED) return PA_ERR_STATE;
    c->sweep_persistent = on != 0;
    if (c->repr != PA_MSC64) return PA_OK;
    drop_graph(c);
    return upload_sweep_plan(c);
}

pa_status pa_set_sweep_chunks(pa_ctx *c, int32_t chunks)
{
    if (!c || chunks < 0 || chunks > MAX_SWEEP_CHUNKS) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED) return PA_ERR_STATE;
    c->sweep_chunks = chunks;
    if (c->repr != PA_MSC64) return PA_OK;
    drop_graph(c);
    return upload_sweep_plan(c);
}

pa_status pa_get_sweep_chunks(pa_ctx *c, int32_t *out)
{
    if (!c || !out) return PA_ERR_ARG;
    int K = 1;
    for (int k = 0; k < c->lc.n_sweep_classes; ++k) K = std::max(K, c->lc.sweep_cls[k].nchunk);
    *out = K;
    return PA_OK;
}

pa_status pa_get_sweep_launches(pa_ctx *c, int32_t *out)
{
    if (!c || !out) return PA_ERR_ARG;
    int n = 0;
    for (int k = 0; k < c->lc.n_sweep_classes; ++k) n += c->lc.sweep_cls[k].count > 0 ? 1 : 0;
    *out = n;
    return PA_OK;
}

pa_status pa_set_pooled(pa_ctx *c, int32_t on)
{
    if (!c || (on != 0 && on != 1)) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    if (c->phase != PH_MEASURED) return PA_ERR_STATE;
    c->sweep_pooled = on != 0;
    if (c->repr != PA_MSC64) return PA_OK;
    drop_graph(c);
    return upload_sweep_plan(c);
}

pa_status pa_get_tuning(pa_ctx *c, int32_t L, int32_t *threads, int32_t *groups_per_wg, int32_t *dense_calls,
                        int32_t *persistent, int32_t *pooled)
{
    if (!c || L < 4 || (L & 1)) return PA_ERR_ARG;
    if (threads) *threads = c->sweep_threads;
    if (groups_per_wg) *groups_per_wg = groups_for(c, L);
    if (dense_calls) *dense_calls = c->sweep_dense;
    if (persistent) *persistent = c->sweep_persistent ? 1 : 0;
    if (pooled) *pooled = c->sweep_pooled ? 1 : 0;
    return PA_OK;
}

pa_status pa_read_stats(pa_ctx *c, uint64_t *host_out)
{
    if (!c || !host_out) return PA_ERR_ARG;
    if (c->failed) return PA_ERR_DEVICE;
    return read_stats(c, host_out);
}

const char *pa_last_error(pa_ctx *c)
{
    if (!c) return "no context";
    return c->last == hipSuccess ? "none" : hipGetErrorString(c->last);
}

pa_status pa_create_static(const pa_run_desc *runs, int32_t n_runs, pa_repr repr, void *hip_stream, pa_ctx **out)
{
    if (!out) return PA_ERR_ARG;
    *out = nullptr;
    size_t need = 0;
    const pa_status st0 = pa_workspace_size(runs, n_runs, repr, &need);
    if (st0 != PA_OK) return st0;
    if (need > STATIC_WS_BYTES) return PA_ERR_NOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PA_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticWs &w = g_static_ws[dev];
    if (!w.ptr) {
        // first use on this device (current): resolve its copy of the array
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PA_ERR_DEVICE;
        w.ptr = (uint8_t *)p;
    }
    if (w.owner) return PA_ERR_STATE;   // one live context per device holds the array
    pa_ctx *c = nullptr;
    const pa_status st = pa_create(runs, n_runs, repr, w.ptr, STATIC_WS_BYTES, hip_stream, &c);
    if (st != PA_OK) return st;
    c->static_dev = dev;
    w.owner = c;
    *out = c;
    return PA_OK;
}

pa_status pa_destroy(pa_ctx *c)
{
    if (!c) return PA_ERR_ARG;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_def) (void)hipGraphDestroy(c->graph_def);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        StaticWs &w = g_static_ws[c->static_dev];
        if (w.owner == c) w.owner = nullptr;
    }
    delete c;
    return PA_OK;
}

}  // extern "C"
