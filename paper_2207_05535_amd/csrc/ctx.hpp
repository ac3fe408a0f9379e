// ctx.hpp -- host-side context of libpa.so: workspace plan, launch state and
// the helpers shared by the C ABI (pa_api.hip), the autotuner
// (pa_autotune.hip) and the serving loop (pa_serve.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "../../include/pa.h"
#include "launch.hpp"
#include "pa_internal.hpp"

namespace pa {

enum Phase { PH_MEASURED = 0, PH_ANNEALED = 1, PH_RESAMPLED = 2, PH_SWEPT = 3 };

// Offsets of buffers inside a device region (256-byte aligned).
struct Planner {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// Per-run buffers, as offsets from the start of the region they live in.
struct RunOff {
    size_t spins[MAX_POP][2], E[MAX_POP][2], fam[MAX_POP][2], r[MAX_POP], C[MAX_POP], parent[MAX_POP],
        P[MAX_POP], part[MAX_POP], partS[MAX_POP], tot64[MAX_POP], base64[MAX_POP], tot32[MAX_POP],
        base32[MAX_POP], qh, jbits, wang, dos;
    int table;
};

// Host-built tables of one (N, schedule): reweighting factors X (exact) and
// x (FP64) per temperature and level, Metropolis thresholds, betas.
struct TableOff {
    size_t X, x, T, beta;
    int N, K;
    const double *beta_src;
};

struct Layout {
    std::vector<RunOff> runs;
    std::vector<TableOff> tables;
    size_t runinfo, popstate, items, chunk_items, obs, dseed, logw, wavg, stats, sweep_items, queue, meas_items,
        sweep_flags;
    size_t qw, famst, wq;   // overlap weights, family statistics, weighted overlap distributions
    int n_items, n_chunk_items, n_meas_items, npop_ctx, Kmax, maxN;
    size_t total;
};

bool desc_ok(const pa_run_desc &d, pa_repr repr);
inline int groups_cap_of(const pa_run_desc &d) { return (d.R_cap + 63) / 64; }
inline int chunks_cap_of(const pa_run_desc &d) { return (d.R_cap + CH - 1) / CH; }
void plan_run_buffers(Planner &P, const pa_run_desc &d, pa_repr repr, RunOff &o);
void plan_table(Planner &P, int N, const pa_run_desc &d, TableOff &T);
Layout plan(const pa_run_desc *runs, int n_runs, pa_repr repr);
void compute_tables(const pa_run_desc &d, int N, std::vector<uint64_t> &X, std::vector<double> &x,
                    std::vector<uint64_t> &T);
// RunInfo of a run whose buffers start at `base` (offsets o) and tables at
// `tbase` (offsets T); records through obs with the given stride/offset.
RunInfo make_runinfo(const pa_run_desc &d, uint8_t *base, const RunOff &o, uint8_t *tbase, const TableOff &T,
                     pa_obs *obs, int obs_stride, int obs_off);
PopState initial_popstate(const pa_run_desc &d);
// LDS ints of the permutation-pairing repair: 2 R_cap of the largest such
// run whose labels (8 bytes per replica) fit the workgroup LDS beside the
// kernel's own, 0 if none does (those runs repair in global memory).
int wang_lds_ints_of(const pa_run_desc *const *runs, int n, int lds_limit);
// theta = infinity: energy draw thresholds [K][N+1] of a run (see pa.h);
// false if the density of states is not available for its L.
bool dos_thresholds(const pa_run_desc &d, std::vector<uint64_t> &out);
// Measure items of one (run, pop): 4 / waves-per-group consecutive groups each.
void meas_items_of(const pa_run_desc &d, int run, int pop, std::vector<SweepItem> &out);
inline int n_meas_items_of(const pa_run_desc &d)
{
    const int gpw = MEAS_WAVES / meas_waves_per_group(d.L * d.L);
    return (groups_cap_of(d) + gpw - 1) / gpw;
}
int default_groups(int L);
// Batched-sweep shape for lattice size L from an autotuner cache file.
bool tuning_from_cache(const char *path, int L, int *threads, int *groups, int *dense, int *persistent,
                       int *pooled);

}  // namespace pa

struct pa_ctx {
    int n_runs = 0;
    pa_repr repr = PA_INT8;
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    pa::Layout lo;
    std::vector<pa_run_desc> descs;
    std::vector<std::vector<double>> betas;
    std::vector<pa::RunInfo> hinfo;
    pa::LaunchCtx lc;
    int i = 0;
    int phase = pa::PH_MEASURED;
    bool failed = false;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
    int lds_limit = 65536;
    int sweep_threads = 512;
    int sweep_dense = 3;                // Philox calls every site makes in lockstep
    bool sweep_persistent = false;      // persistent grid with a ticket queue
    bool sweep_pooled = false;          // sparse rounds over one list per workgroup
    int sweep_chunks = 1;               // chunks of sweeps per item on the persistent grid, 0: chosen per plan
    std::map<int, int> groups_per_wg;   // L -> replica groups per workgroup of the batched sweep
    bool any_multinomial = false;
    bool any_wang = false;
    bool any_exact_dos = false;
    hipError_t last = hipSuccess;
    int static_dev = -1;                // device whose static workspace this context holds, or -1
};

namespace pa {

template <typename T>
T *at(pa_ctx *c, size_t off)
{
    return (T *)(c->ws + off);
}

pa_status dev_fail(pa_ctx *c, hipError_t e = hipSuccess);

#define PA_HIP(ctx, expr)                                  \
    do {                                                   \
        const hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return dev_fail(ctx, e_);    \
    } while (0)

int groups_for(const pa_ctx *c, int L);
bool plan_sweep(const pa_ctx *c, std::vector<SweepItem> &items, size_t &lds);
pa_status upload_sweep_plan(pa_ctx *c);
pa_status enqueue_step(pa_ctx *c);
void drop_graph(pa_ctx *c);
pa_status read_stats(pa_ctx *c, uint64_t out[3]);   // sums the counter slots; synchronises

}  // namespace pa
