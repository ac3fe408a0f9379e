// launch.hpp -- host-side launchers of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "pa_internal.hpp"

namespace pa {

// One launch of the batched sweep: the items of one (lattice size, model)
// class, swept by the kernel compiled for that class (L = 0: the kernel
// that dispatches per item, for the sizes without one of their own).
struct SweepClass {
    int first, count;   // items [first, first + count) of the sweep list
    int L, ea;
    int grid;           // > 0: persistent grid of this many workgroups
    size_t lds;
    int nchunk = 1;     // > 1: items split into this many chunks of sweeps (persistent grid only)
};
constexpr int MAX_SWEEP_CLASSES = 16;

struct LaunchCtx {
    const RunInfo *runs;      // device [n_runs]
    PopState *st;             // device [n_runs][MAX_POP]
    const Item *items;        // device [n_items]: every (run, pop, group < groups_cap)
    int n_items;
    const ChunkItem *chunk_items;  // device: every (run, pop, chunk < chunks_cap)
    int n_chunk_items;
    int run0, n_runs, npop_ctx;    // per-run launches cover runs [run0, run0 + n_runs)
    int repr;
    bool any_multinomial;
    bool any_overlap = true;       // some run measures overlaps (index shift, two populations, pairing)
    int mn_split = CH_PER;         // workgroups per chunk of multinomial draws: CH_PER if a run spans chunks, else 1
    int copy_split = 1;            // workgroups per copy item, each taking a share of every group's 64-site blocks
    bool any_wang;                 // some run pairs replicas by permutations
    int wang_lds_ints;             // LDS of the pairing repair (2 R_cap of the largest run that fits, or 0)
    bool any_exact_dos;            // some run is at theta = infinity
    unsigned long long *stats;   // device [NSTAT] work counters of the sweeps
    const SweepItem *meas_items;   // device [n_meas_items]: groups per measure workgroup
    int n_meas_items;
    const SweepItem *sweep_items;  // device [n_sweep_items], grouped by class
    int n_sweep_items, sweep_threads, sweep_dense;
    int sweep_pooled;              // 1: sparse rounds over one list per workgroup
    int n_sweep_classes = 0;       // launches of the batched sweep, one per class
    SweepClass sweep_cls[MAX_SWEEP_CLASSES];
    unsigned int *sweep_queue;     // device [4]: ticket counters of the persistent grid, launch generation
    unsigned int *sweep_flags = nullptr;   // device [n_items]: completed sweep chunk of each item's groups
    hipStream_t stream;
};

hipError_t launch_fill_u32(void *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_init(const LaunchCtx &c, const uint64_t *dseed);
hipError_t launch_anneal(const LaunchCtx &c);
hipError_t launch_resample(const LaunchCtx &c);
hipError_t launch_sweep_int8_run(const LaunchCtx &c, int run, int L, int groups_cap, int npop, int theta);
hipError_t launch_sweep_msc(const LaunchCtx &c);
hipError_t launch_measure(const LaunchCtx &c);
hipError_t launch_dos_sample(const LaunchCtx &c);   // theta = infinity draws (no-op without such runs)
hipError_t launch_wavg(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K, int i_done,
                       double *logw, double *qw, pa_wavg *out);
hipError_t launch_qweights(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K, int i_done,
                           double *logw, double *qw);
hipError_t launch_wqhist(const LaunchCtx &c, const pa_obs *obs, int M, int kind, int pop, int K, int i_done,
                         double *logw, double *qw, double *out);
hipError_t launch_famstats(const LaunchCtx &c, const pa_obs *obs, int pop, int K, int i_done, pa_famstat *out);
int int8_tile_rows(int L);
// LDS bytes of a batched-sweep workgroup of `threads` holding `groups`
// replica groups of N sites (ea: the spin glass), launched with mode =
// lockstep calls | pooled << 8.
size_t msc_lds_bytes(int N, int groups, bool ea, int threads, int mode);
hipError_t prepare_msc_lds(size_t bytes);
int sweep_msc_resident(int threads, size_t lds, int L, int ea);   // workgroups resident on the device, 0 on error
bool msc_specialised(int L);   // a sweep kernel compiled for this L alone exists
// The launches of the batched sweep for these items (already largest
// first): drops the items of runs without Metropolis sweeps (run_L[r] = 0:
// theta = 0 or the theta = infinity limit) and fills cls with the classes
// to launch (run_L[r], run_ea[r]: run r's lattice size and model).  Returns
// the number of classes (at most MAX_SWEEP_CLASSES), or -1 on error.
// threads and mode: the launch's workgroup size and mode (msc_lds_bytes).
// split_ok: mixed sizes may get one launch per size when every class fills
// the chip (this queries occupancy: the LDS limit must already be set).
int sweep_classes(std::vector<SweepItem> &items, const std::vector<int> &run_L, const std::vector<int> &run_ea,
                  SweepClass *cls, int threads, int mode, bool split_ok);
// Persistent grids of the classes (threads per workgroup as launched).
bool sweep_class_grids(SweepClass *cls, int n, int threads, bool persistent);
// Chunks of sweeps per item for a persistent launch of n items on `slots`
// resident workgroups: 1 when every item gets a workgroup at once, else the
// count that least quantises the launch into rounds.
int sweep_chunks_auto(int n, int slots);
// Replaces the (single) class's items by K chunks of each, all first chunks
// first, with the sweeps of each chunk (run_theta[r]: run r's theta); 0 on
// success, -1 if the class does not cover the whole list.
int expand_sweep_chunks(std::vector<SweepItem> &items, SweepClass &cls, int K, const std::vector<int> &run_theta);
hipError_t prepare_wang_lds(size_t bytes);
hipError_t launch_philox_rate(int calls, hipStream_t s, int *blocks, int *threads);

}  // namespace pa
