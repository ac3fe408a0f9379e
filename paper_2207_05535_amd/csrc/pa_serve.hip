// pa_serve.hip -- continuous batching of independent PA runs on one GPU.
//
// A server owns one device arena (caller-allocated) and a fixed table of
// slots.  Each admitted run gets a contiguous block of the arena for its
// populations, records and work lists; runs with the same lattice size and
// temperature schedule share one block of host-built tables (reference
// counted).  Admission is by footprint: a run is admitted only if a slot is
// free and its block fits in the free space of the arena (first fit, with
// coalescing of freed blocks), otherwise the caller is told to retry later.
//
// One server step advances every resident run that has not reached its
// last temperature by one temperature step (Sec. II B steps ii-v), whatever
// temperature each run is at: every kernel reads a run's temperature index
// from its own device state.  All resident runs share the launches of a
// step (one sweep launch covers every run's lattice blocks), so runs
// admitted while others are in flight overlap with them on the device.  A
// run's results depend only on its descriptor: the same records come out
// alone or in any mix.
//
// Everything is enqueued on the caller's stream in order, so memory released
// by a finished run can be handed to a new run at once: the new run's
// initialisation runs after all earlier work on that memory.  Host data for
// uploads is kept alive until an event recorded after its copy has passed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "ctx.hpp"

using namespace pa;

namespace {

// First-fit allocator over [start, end) with coalescing; 256-byte granules.
class Arena {
public:
    void reset(size_t start, size_t end)
    {
        free_.clear();
        const size_t a = (start + 255) & ~(size_t)255, b = end & ~(size_t)255;
        if (b > a) free_[a] = b - a;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;   // offset -> length
    size_t used_ = 0;
};

// Per-run block: buffers of plan_run_buffers, then records, work lists and
// the disorder seed.
struct BlockPlan {
    RunOff o;
    size_t obs, items, chunks, meas, dseed, bytes;
};

BlockPlan plan_block(const pa_run_desc &d, pa_repr repr)
{
    BlockPlan b;
    Planner P;
    plan_run_buffers(P, d, repr, b.o);
    const int npop = n_pop_of(d.overlap);
    b.obs = P.take(sizeof(pa_obs) * (size_t)d.K * npop);
    b.items = P.take(sizeof(Item) * (size_t)npop * groups_cap_of(d));
    b.chunks = P.take(sizeof(ChunkItem) * (size_t)npop * chunks_cap_of(d));
    b.meas = P.take(sizeof(SweepItem) * (size_t)npop * n_meas_items_of(d));
    b.dseed = P.take(sizeof(uint64_t));
    b.bytes = P.off;
    return b;
}

size_t table_bytes(const pa_run_desc &d)
{
    Planner P;
    TableOff T;
    plan_table(P, d.L * d.L, d, T);
    return P.off;
}

struct Table {
    int N = 0, K = 0, refs = 0;
    std::vector<double> beta;
    TableOff T;       // offsets relative to `off`
    size_t off = 0, bytes = 0;   // block in the arena
};

struct Slot {
    bool used = false;
    pa_run_desc d;
    std::vector<double> beta;
    BlockPlan b;
    size_t off = 0;      // block offset from the arena start
    int table = -1;
    int done = 0;        // temperature index reached (as enqueued)
};

struct Upload {
    hipEvent_t ev;
    std::vector<uint8_t> data;
};

}  // namespace

struct pa_server {
    pa_repr repr = PA_MSC64;
    hipStream_t stream = nullptr;
    uint8_t *base = nullptr;
    size_t bytes = 0;
    int max_slots = 0;
    size_t runinfo = 0, popstate = 0, stats = 0, queue = 0, header = 0;
    Arena arena;
    std::vector<Slot> slots;
    std::vector<Table> tables;
    // batch work lists in the arena (grown on demand)
    size_t items_off = 0, items_cap = 0, chunks_off = 0, chunks_cap = 0, sweep_off = 0, sweep_cap = 0;
    size_t meas_off = 0, meas_cap = 0;
    bool dirty = true;
    LaunchCtx lc;
    std::deque<Upload> pending;
    int lds_limit = 65536;
    int threads = 512, dense = 3;
    bool persistent = false, pooled = false;
    std::map<int, int> groups;
    bool failed = false;
    hipError_t last = hipSuccess;
};

namespace {

pa_status sfail(pa_server *s, hipError_t e = hipSuccess)
{
    s->failed = true;
    if (e == hipSuccess) e = hipGetLastError();
    if (s->last == hipSuccess) s->last = e;
    return PA_ERR_DEVICE;
}

#define PA_SHIP(srv, expr)                                  \
    do {                                                    \
        const hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return sfail(srv, e_);        \
    } while (0)

void reap(pa_server *s)
{
    while (!s->pending.empty() && hipEventQuery(s->pending.front().ev) == hipSuccess) {
        (void)hipEventDestroy(s->pending.front().ev);
        s->pending.pop_front();
    }
}

pa_status upload(pa_server *s, void *dst, const void *src, size_t n)
{
    if (n == 0) return PA_OK;
    Upload u;
    u.data.assign((const uint8_t *)src, (const uint8_t *)src + n);
    PA_SHIP(s, hipMemcpyAsync(dst, u.data.data(), n, hipMemcpyHostToDevice, s->stream));
    PA_SHIP(s, hipEventCreateWithFlags(&u.ev, hipEventDisableTiming));
    const hipError_t e = hipEventRecord(u.ev, s->stream);
    s->pending.push_back(std::move(u));
    if (e != hipSuccess) return sfail(s, e);
    return PA_OK;
}

// The batched sweep's launch mode: lockstep calls | pooled << 8.
int serve_mode(const pa_server *s)
{
    return s->dense | (s->pooled ? 1 << 8 : 0);
}

int groups_of(const pa_server *s, int L)
{
    auto it = s->groups.find(L);
    return it == s->groups.end() ? default_groups(L) : it->second;
}

// Regrows a work-list region to hold `need` bytes (doubling).  The old
// region is released at once: later users of that memory are enqueued after
// every launch that read the old list.
bool grow(pa_server *s, size_t &off, size_t &cap, size_t need)
{
    if (need <= cap) return true;
    size_t ncap = std::max(need, 2 * cap);
    size_t noff = 0;
    if (!s->arena.alloc(ncap, &noff)) {
        ncap = need;
        if (!s->arena.alloc(ncap, &noff)) return false;
    }
    if (cap) s->arena.release(off, cap);
    off = noff;
    cap = ncap;
    return true;
}

// Batch work lists of every resident run: the per-run lists are copied
// device to device into one array each; the sweep items (largest lattice
// block first) are built on the host.
pa_status rebuild(pa_server *s)
{
    size_t n_items = 0, n_chunks = 0, n_meas = 0;
    int hi = 0, npop_ctx = 1;
    bool mn = false, wang = false, exact = false, mn_wide = false, ovl = false;
    std::vector<SweepItem> sweep;
    size_t lds = 0;
    for (int k = 0; k < s->max_slots; ++k) {
        const Slot &sl = s->slots[k];
        if (!sl.used) continue;
        const int npop = n_pop_of(sl.d.overlap);
        n_items += (size_t)npop * groups_cap_of(sl.d);
        n_chunks += (size_t)npop * chunks_cap_of(sl.d);
        n_meas += (size_t)npop * n_meas_items_of(sl.d);
        hi = k + 1;
        npop_ctx = std::max(npop_ctx, npop);
        mn = mn || sl.d.resampling == PA_MULTINOMIAL;
        mn_wide = mn_wide || (sl.d.resampling == PA_MULTINOMIAL && sl.d.R > CH);
        ovl = ovl || sl.d.overlap != PA_Q_NONE;
        wang = wang || is_wang(sl.d.overlap);
        exact = exact || sl.d.theta == PA_THETA_EXACT;
        if (s->repr == PA_MSC64) {
            const int G = groups_of(s, sl.d.L);
            const int N = sl.d.L * sl.d.L;
            if ((size_t)G * N > 65535) return PA_ERR_ARG;
            lds = std::max(lds, msc_lds_bytes(N, G, sl.d.model == PA_EA_PMJ, s->threads,
                                              serve_mode(s) | MSC_WHOLE_LISTS));
            for (int p = 0; p < npop; ++p)
                for (int g = 0; g < groups_cap_of(sl.d); g += G)
                    sweep.push_back({k, p, g, std::min(G, groups_cap_of(sl.d) - g)});
        }
    }
    if (lds > (size_t)s->lds_limit) return PA_ERR_ARG;
    std::stable_sort(sweep.begin(), sweep.end(), [s](const SweepItem &a, const SweepItem &b) {
        const long wa = (long)a.ngroups * s->slots[a.run].d.L * s->slots[a.run].d.L;
        const long wb = (long)b.ngroups * s->slots[b.run].d.L * s->slots[b.run].d.L;
        return wa > wb;
    });
    // lattice size and model of each slot's run, for the per-class sweep launches
    std::vector<int> run_L(std::max(hi, 1), 0), run_ea(std::max(hi, 1), 0);
    for (int k = 0; k < hi; ++k)
        if (s->slots[k].used) {
            run_L[k] = s->slots[k].d.theta > 0 ? s->slots[k].d.L : 0;
            run_ea[k] = s->slots[k].d.model == PA_EA_PMJ;
        }
    if (s->repr == PA_MSC64) {
        SweepClass probe[MAX_SWEEP_CLASSES];
        // orders the list by class; a serving mix keeps one launch for its
        // sizes (their classes are too small to fill the chip one by one)
        if (sweep_classes(sweep, run_L, run_ea, probe, s->threads, serve_mode(s), false) < 0)
            return PA_ERR_ARG;
    }
    if (!grow(s, s->items_off, s->items_cap, sizeof(Item) * std::max<size_t>(n_items, 1)) ||
        !grow(s, s->chunks_off, s->chunks_cap, sizeof(ChunkItem) * std::max<size_t>(n_chunks, 1)) ||
        !grow(s, s->sweep_off, s->sweep_cap, sizeof(SweepItem) * std::max<size_t>(sweep.size(), 1)) ||
        !grow(s, s->meas_off, s->meas_cap, sizeof(SweepItem) * std::max<size_t>(n_meas, 1)))
        return PA_ERR_NOMEM;
    size_t ai = 0, ac = 0, am = 0;
    for (int k = 0; k < s->max_slots; ++k) {
        const Slot &sl = s->slots[k];
        if (!sl.used) continue;
        const int npop = n_pop_of(sl.d.overlap);
        const size_t ni = (size_t)npop * groups_cap_of(sl.d), nc = (size_t)npop * chunks_cap_of(sl.d);
        const size_t nm = (size_t)npop * n_meas_items_of(sl.d);
        uint8_t *blk = s->base + sl.off;
        PA_SHIP(s, hipMemcpyAsync(s->base + s->items_off + ai * sizeof(Item), blk + sl.b.items, ni * sizeof(Item),
                                  hipMemcpyDeviceToDevice, s->stream));
        PA_SHIP(s, hipMemcpyAsync(s->base + s->chunks_off + ac * sizeof(ChunkItem), blk + sl.b.chunks,
                                  nc * sizeof(ChunkItem), hipMemcpyDeviceToDevice, s->stream));
        PA_SHIP(s, hipMemcpyAsync(s->base + s->meas_off + am * sizeof(SweepItem), blk + sl.b.meas,
                                  nm * sizeof(SweepItem), hipMemcpyDeviceToDevice, s->stream));
        ai += ni;
        ac += nc;
        am += nm;
    }
    pa_status st = upload(s, s->base + s->sweep_off, sweep.data(), sizeof(SweepItem) * sweep.size());
    if (st != PA_OK) return st;
    LaunchCtx &c = s->lc;
    c.items = (const Item *)(s->base + s->items_off);
    c.n_items = (int)n_items;
    c.chunk_items = (const ChunkItem *)(s->base + s->chunks_off);
    c.n_chunk_items = (int)n_chunks;
    c.meas_items = (const SweepItem *)(s->base + s->meas_off);
    c.n_meas_items = (int)n_meas;
    c.run0 = 0;
    c.n_runs = hi;
    c.npop_ctx = npop_ctx;
    c.any_multinomial = mn;
    c.mn_split = mn_wide ? CH_PER : 1;
    c.copy_split = 1;   // requests of any size share the copy launch
    c.any_overlap = ovl;
    c.any_wang = wang;
    {
        std::vector<const pa_run_desc *> dp;
        for (int k = 0; k < s->max_slots; ++k)
            if (s->slots[k].used) dp.push_back(&s->slots[k].d);
        c.wang_lds_ints = wang_lds_ints_of(dp.data(), (int)dp.size(), s->lds_limit);
        if (c.wang_lds_ints && prepare_wang_lds(sizeof(int32_t) * (size_t)c.wang_lds_ints) != hipSuccess)
            return sfail(s);
    }
    c.any_exact_dos = exact;
    c.sweep_items = (const SweepItem *)(s->base + s->sweep_off);
    c.n_sweep_items = (int)sweep.size();
    c.sweep_threads = s->threads;
    c.sweep_dense = s->dense;
    c.sweep_pooled = s->pooled ? 1 : 0;
    c.n_sweep_classes = 0;
    if (s->repr == PA_MSC64 && !sweep.empty()) {
        if (prepare_msc_lds(lds) != hipSuccess) return sfail(s);
        const int ncls = sweep_classes(sweep, run_L, run_ea, c.sweep_cls, s->threads, serve_mode(s), false);
        if (ncls < 0) return PA_ERR_ARG;
        if (!sweep_class_grids(c.sweep_cls, ncls, s->threads, s->persistent)) return sfail(s);
        c.n_sweep_classes = ncls;
        c.n_sweep_items = (int)sweep.size();
    }
    s->dirty = false;
    return PA_OK;
}

void release_table(pa_server *s, int t)
{
    Table &T = s->tables[t];
    if (--T.refs == 0) {
        s->arena.release(T.off, T.bytes);
        T.beta.clear();
        T.N = T.K = 0;
    }
}

}  // namespace

extern "C" {

pa_status pa_server_footprint(const pa_run_desc *desc, pa_repr repr, size_t *bytes)
{
    if (!desc || !bytes || (repr != PA_INT8 && repr != PA_MSC64) || !desc_ok(*desc, repr)) return PA_ERR_ARG;
    *bytes = plan_block(*desc, repr).bytes + table_bytes(*desc);
    return PA_OK;
}

pa_status pa_server_create(pa_repr repr, void *dev_arena, size_t arena_bytes, int32_t max_slots,
                           const char *tuning_cache, void *hip_stream, pa_server **out)
{
    if (!out) return PA_ERR_ARG;
    *out = nullptr;
    if ((repr != PA_INT8 && repr != PA_MSC64) || !dev_arena || ((uintptr_t)dev_arena & 255) || max_slots < 1 ||
        max_slots > 65536)
        return PA_ERR_ARG;
    Planner P;
    const size_t runinfo = P.take(sizeof(RunInfo) * max_slots);
    const size_t popstate = P.take(sizeof(PopState) * max_slots * MAX_POP);
    const size_t stats = P.take(STAT_BYTES);
    const size_t queue = P.take(sizeof(uint32_t) * 4);
    if (arena_bytes < P.off + 4096) return PA_ERR_NOMEM;

    pa_server *s = new pa_server();
    s->repr = repr;
    s->stream = (hipStream_t)hip_stream;
    s->base = (uint8_t *)dev_arena;
    s->bytes = arena_bytes;
    s->max_slots = max_slots;
    s->runinfo = runinfo;
    s->popstate = popstate;
    s->stats = stats;
    s->queue = queue;
    s->header = P.off;
    s->slots.resize(max_slots);
    // the header is never handed out: the allocator covers the rest
    s->arena.reset(s->header, arena_bytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&s->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        delete s;
        return PA_ERR_DEVICE;
    }
    if (tuning_cache) {
        int th = 0, g = 0, dn = 0, pe = 0, po = 0;
        for (int L = 4; L <= 128; L += 2)
            if (tuning_from_cache(tuning_cache, L, &th, &g, &dn, &pe, &po)) {
                s->groups[L] = g;
                if (L == 64 || s->groups.size() == 1) {   // shared knobs: from L = 64 when present
                    s->threads = th;
                    s->dense = dn;
                    s->persistent = pe != 0;
                    s->pooled = po != 0;
                }
            }
    }
    LaunchCtx &c = s->lc;
    std::memset(&c, 0, sizeof(c));
    c.runs = (const RunInfo *)(s->base + runinfo);
    c.st = (PopState *)(s->base + popstate);
    c.repr = repr;
    c.stats = (unsigned long long *)(s->base + stats);
    c.sweep_queue = (unsigned int *)(s->base + queue);
    c.stream = s->stream;
    bool ok = launch_fill_u32(s->base, 0, s->header / 4, s->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(s->stream) == hipSuccess;
    if (!ok) {
        delete s;
        return PA_ERR_DEVICE;
    }
    *out = s;
    return PA_OK;
}

pa_status pa_server_admit(pa_server *s, const pa_run_desc *desc, int32_t *slot)
{
    if (!s || !desc || !slot || !desc_ok(*desc, s->repr)) return PA_ERR_ARG;
    if (s->failed) return PA_ERR_DEVICE;
    reap(s);
    int k = 0;
    while (k < s->max_slots && s->slots[k].used) ++k;
    if (k == s->max_slots) return PA_ERR_CAPACITY;
    const pa_run_desc &d = *desc;
    if (s->repr == PA_MSC64) {
        const int N = d.L * d.L, G = groups_of(s, d.L);
        if ((size_t)G * N > 65535 ||
            msc_lds_bytes(N, G, d.model == PA_EA_PMJ, s->threads, serve_mode(s) | MSC_WHOLE_LISTS) >
                (size_t)s->lds_limit)
            return PA_ERR_ARG;
    }
    const int N = d.L * d.L;
    int t = -1;
    for (size_t q = 0; q < s->tables.size(); ++q) {
        const Table &T = s->tables[q];
        if (T.refs > 0 && T.N == N && T.K == d.K && std::memcmp(T.beta.data(), d.beta, sizeof(double) * d.K) == 0)
            t = (int)q;
    }
    Slot &sl = s->slots[k];
    const BlockPlan b = plan_block(d, s->repr);
    size_t off = 0;
    if (!s->arena.alloc(b.bytes, &off)) return PA_ERR_NOMEM;
    bool new_table = false;
    if (t < 0) {
        Table T;
        T.N = N;
        T.K = d.K;
        T.beta.assign(d.beta, d.beta + d.K);
        Planner P;
        pa_run_desc dd = d;
        dd.beta = T.beta.data();
        plan_table(P, N, dd, T.T);
        T.bytes = P.off;
        if (!s->arena.alloc(T.bytes, &T.off)) {
            s->arena.release(off, b.bytes);
            return PA_ERR_NOMEM;
        }
        for (size_t q = 0; q < s->tables.size() && t < 0; ++q)
            if (s->tables[q].refs == 0) t = (int)q;
        if (t < 0) {
            s->tables.push_back(Table());
            t = (int)s->tables.size() - 1;
        }
        s->tables[t] = std::move(T);
        new_table = true;
    }
    Table &T = s->tables[t];
    T.refs += 1;
    sl.used = true;
    sl.d = d;
    sl.beta.assign(d.beta, d.beta + d.K);
    sl.d.beta = sl.beta.data();
    sl.b = b;
    sl.off = off;
    sl.table = t;
    sl.done = 0;

    uint8_t *blk = s->base + off;
    uint8_t *tbase = s->base + T.off;
    pa_status st = PA_OK;
    if (new_table) {
        std::vector<uint64_t> X, TT;
        std::vector<double> x;
        compute_tables(sl.d, N, X, x, TT);
        if ((st = upload(s, tbase + T.T.X, X.data(), sizeof(uint64_t) * X.size())) != PA_OK ||
            (st = upload(s, tbase + T.T.x, x.data(), sizeof(double) * x.size())) != PA_OK ||
            (st = upload(s, tbase + T.T.T, TT.data(), sizeof(uint64_t) * TT.size())) != PA_OK ||
            (st = upload(s, tbase + T.T.beta, T.beta.data(), sizeof(double) * d.K)) != PA_OK)
            return st;
    }
    const int npop = n_pop_of(d.overlap);
    const RunInfo I = make_runinfo(sl.d, blk, b.o, tbase, T.T, (pa_obs *)(blk + b.obs), npop, 0);
    PopState hst[MAX_POP];
    std::memset(hst, 0, sizeof(hst));
    for (int p = 0; p < npop; ++p) hst[p] = initial_popstate(sl.d);
    std::vector<Item> items;
    std::vector<ChunkItem> chunks;
    std::vector<SweepItem> meas;
    for (int p = 0; p < npop; ++p) {
        for (int g = 0; g < groups_cap_of(d); ++g) items.push_back({k, p, g, 0});
        for (int q = 0; q < chunks_cap_of(d); ++q) chunks.push_back({k, p, q, 0});
        meas_items_of(d, k, p, meas);
    }
    const uint64_t ds = d.disorder_seed;
    if ((st = upload(s, s->base + s->runinfo + sizeof(RunInfo) * k, &I, sizeof(I))) != PA_OK ||
        (st = upload(s, s->base + s->popstate + sizeof(PopState) * MAX_POP * k, hst, sizeof(hst))) != PA_OK ||
        (st = upload(s, blk + b.items, items.data(), sizeof(Item) * items.size())) != PA_OK ||
        (st = upload(s, blk + b.chunks, chunks.data(), sizeof(ChunkItem) * chunks.size())) != PA_OK ||
        (st = upload(s, blk + b.meas, meas.data(), sizeof(SweepItem) * meas.size())) != PA_OK ||
        (st = upload(s, blk + b.dseed, &ds, sizeof(ds))) != PA_OK)
        return st;
    if (d.theta == PA_THETA_EXACT) {   // energy draw thresholds of the theta = infinity limit
        std::vector<uint64_t> D;
        if (!dos_thresholds(sl.d, D)) return PA_ERR_ARG;
        if ((st = upload(s, blk + b.o.dos, D.data(), sizeof(uint64_t) * D.size())) != PA_OK) return st;
    }
    bool ok = true;
    for (int p = 0; p < npop && ok; ++p) ok = launch_fill_u32(blk + b.o.r[p], 0, d.R_cap, s->stream) == hipSuccess;
    if (d.qhist && ok)
        ok = launch_fill_u32(blk + b.o.qh, 0, (size_t)npop * d.K * (N + 1), s->stream) == hipSuccess;
    ok = ok && launch_fill_u32(blk + b.obs, 0, sizeof(pa_obs) / 4 * (size_t)d.K * npop, s->stream) == hipSuccess;
    if (!ok) return sfail(s);
    // step (i) and the measurement at i = 0, for this run only
    LaunchCtx c = s->lc;
    c.items = (const Item *)(blk + b.items);
    c.n_items = (int)items.size();
    c.chunk_items = (const ChunkItem *)(blk + b.chunks);
    c.n_chunk_items = (int)chunks.size();
    c.meas_items = (const SweepItem *)(blk + b.meas);
    c.n_meas_items = (int)meas.size();
    c.run0 = k;
    c.n_runs = 1;
    c.npop_ctx = npop;
    c.any_multinomial = d.resampling == PA_MULTINOMIAL;
    c.mn_split = d.resampling == PA_MULTINOMIAL && d.R > CH ? CH_PER : 1;
    c.any_overlap = d.overlap != PA_Q_NONE;
    c.any_wang = is_wang(d.overlap);
    {
        const pa_run_desc *dp = &sl.d;
        c.wang_lds_ints = wang_lds_ints_of(&dp, 1, s->lds_limit);
        if (c.wang_lds_ints && prepare_wang_lds(sizeof(int32_t) * (size_t)c.wang_lds_ints) != hipSuccess)
            return sfail(s);
    }
    c.any_exact_dos = d.theta == PA_THETA_EXACT;
    if (launch_init(c, (const uint64_t *)(blk + b.dseed)) != hipSuccess || launch_measure(c) != hipSuccess)
        return sfail(s);
    s->dirty = true;
    *slot = k;
    return PA_OK;
}

pa_status pa_server_step(pa_server *s, int32_t *finished, int32_t *n_finished)
{
    if (!s || !finished || !n_finished) return PA_ERR_ARG;
    *n_finished = 0;
    if (s->failed) return PA_ERR_DEVICE;
    reap(s);
    bool any = false;
    for (const Slot &sl : s->slots)
        if (sl.used && sl.done < sl.d.K - 1) any = true;
    if (!any) return PA_OK;
    pa_status st;
    if (s->dirty && (st = rebuild(s)) != PA_OK) return st;
    const LaunchCtx &c = s->lc;
    hipError_t e = launch_anneal(c);
    if (e == hipSuccess) e = launch_resample(c);
    if (e != hipSuccess) return sfail(s, e);
    if (s->repr == PA_MSC64) {
        if ((e = launch_sweep_msc(c)) != hipSuccess) return sfail(s, e);
    } else {
        for (int k = 0; k < s->max_slots; ++k) {
            const Slot &sl = s->slots[k];
            if (!sl.used || sl.done >= sl.d.K - 1) continue;
            if (launch_sweep_int8_run(c, k, sl.d.L, groups_cap_of(sl.d), n_pop_of(sl.d.overlap), sl.d.theta) !=
                hipSuccess)
                return sfail(s);
        }
    }
    if ((e = launch_dos_sample(c)) != hipSuccess) return sfail(s, e);
    if ((e = launch_measure(c)) != hipSuccess) return sfail(s, e);
    for (int k = 0; k < s->max_slots; ++k) {
        Slot &sl = s->slots[k];
        if (!sl.used || sl.done >= sl.d.K - 1) continue;
        if (++sl.done == sl.d.K - 1) finished[(*n_finished)++] = k;
    }
    return PA_OK;
}

pa_status pa_server_progress(pa_server *s, int32_t slot, int32_t *i_done)
{
    if (!s || !i_done || slot < 0 || slot >= s->max_slots || !s->slots[slot].used) return PA_ERR_ARG;
    *i_done = s->slots[slot].done;
    return PA_OK;
}

pa_status pa_server_read_obs(pa_server *s, int32_t slot, pa_obs *host_out, int32_t sync)
{
    if (!s || !host_out || slot < 0 || slot >= s->max_slots || !s->slots[slot].used || (sync != 0 && sync != 1))
        return PA_ERR_ARG;
    if (s->failed) return PA_ERR_DEVICE;
    const Slot &sl = s->slots[slot];
    const size_t n = (size_t)sl.d.K * n_pop_of(sl.d.overlap);
    PA_SHIP(s, hipMemcpyAsync(host_out, s->base + sl.off + sl.b.obs, sizeof(pa_obs) * n, hipMemcpyDeviceToHost,
                              s->stream));
    if (sync) PA_SHIP(s, hipStreamSynchronize(s->stream));
    return PA_OK;
}

pa_status pa_server_release(pa_server *s, int32_t slot)
{
    if (!s || slot < 0 || slot >= s->max_slots || !s->slots[slot].used) return PA_ERR_ARG;
    if (s->failed) return PA_ERR_DEVICE;
    Slot &sl = s->slots[slot];
    // an empty RunInfo (no populations) makes every per-run kernel skip the slot
    RunInfo empty;
    std::memset(&empty, 0, sizeof(empty));
    pa_status st = upload(s, s->base + s->runinfo + sizeof(RunInfo) * slot, &empty, sizeof(empty));
    if (st != PA_OK) return st;
    s->arena.release(sl.off, sl.b.bytes);
    release_table(s, sl.table);
    sl.used = false;
    sl.table = -1;
    s->dirty = true;
    return PA_OK;
}

pa_status pa_server_info(pa_server *s, int32_t *resident, size_t *bytes_used, size_t *largest_free)
{
    if (!s) return PA_ERR_ARG;
    int n = 0;
    for (const Slot &sl : s->slots) n += sl.used ? 1 : 0;
    if (resident) *resident = n;
    if (bytes_used) *bytes_used = s->arena.used();
    if (largest_free) *largest_free = s->arena.largest();
    return PA_OK;
}

const char *pa_server_last_error(pa_server *s)
{
    if (!s) return "no server";
    return s->last == hipSuccess ? "none" : hipGetErrorString(s->last);
}

pa_status pa_server_destroy(pa_server *s)
{
    if (!s) return PA_ERR_ARG;
    (void)hipStreamSynchronize(s->stream);
    while (!s->pending.empty()) {
        (void)hipEventDestroy(s->pending.front().ev);
        s->pending.pop_front();
    }
    delete s;
    return PA_OK;
}

}  // extern "C"
