// launch.hpp -- host-side launchers of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "pa_internal.hpp"

namespace pa {

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
    bool any_wang;                 // some run pairs replicas by permutations
    int wang_lds_ints;             // LDS of the pairing repair (2 R_cap of the largest run that fits, or 0)
    bool any_exact_dos;            // some run is at theta = infinity
    unsigned long long *stats;   // device [NSTAT] work counters of the sweeps
    const SweepItem *meas_items;   // device [n_meas_items]: groups per measure workgroup
    int n_meas_items;
    const SweepItem *sweep_items;  // device [n_sweep_items]
    int n_sweep_items, sweep_threads, sweep_dense;
    int sweep_grid;                // > 0: persistent grid of this many workgroups
    int sweep_pooled;              // 1: sparse rounds over one list per workgroup
    int sweep_L = 0, sweep_ea = 0;  // every run of the context has this L and model (0: mixed)
    unsigned int *sweep_queue;     // device [2] ticket counters of the persistent grid
    size_t sweep_lds;
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
size_t msc_lds_bytes(int N, int groups);
hipError_t prepare_msc_lds(size_t bytes);
int sweep_msc_resident(int threads, size_t lds, int L, int ea);   // workgroups resident on the device, 0 on error
bool msc_specialised(int L);   // a sweep kernel compiled for this L alone exists
hipError_t prepare_wang_lds(size_t bytes);
hipError_t launch_philox_rate(int calls, hipStream_t s, int *blocks, int *threads);

}  // namespace pa
