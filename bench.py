#!/usr/bin/env python3
"""Spin flips per nanosecond of population annealing on one MI355X.

Workload: 2D Ising ferromagnet, L = 64 periodic, R = 100000 replicas,
beta linear 0 -> 0.6 in 200 points (199 temperature steps), theta = 10
checkerboard Metropolis sweeps per temperature, multinomial resampling,
seeded synthetic initial states.

One "step" is one temperature step of the whole hot path: reweighting and
ln Q (step ii), resampling with contiguous copies (step iii), theta sweeps
(step iv) and measurement (step v); the timed region ends with the FP64
weighted average over the runs (Sec. IV).  Flips = attempted single-spin
updates, sum over steps of theta * R_i * N.

Headline value: the batched path (64 replicas bit-packed per word, lattice
held in LDS for all theta sweeps, every kernel of a step captured in one HIP
graph and replayed; launch shapes from the autotuner).  Reported beside it:
the plain path (int8 spins, one colour of one run per launch, host-driven
steps) on the same workload, whose records must equal the batched path's bit
for bit; the dominant kernel's ALU roofline; and the CPU oracle on a bounded
sample.

Further workloads in the same JSON line (skipped with --quick):
  two_pop_ea   EA +-J, L = 32, two populations of R = 200000 on one
               disorder sample, beta 0 -> 3 in 301 points, theta = 10,
               overlaps q and link overlaps between the populations;
  batched_4096 4096 independent FM runs, L in {8, 16, 24, 32} (1024 each),
               R = 2000, beta 0 -> 0.6 in 150 points, theta = 10, all in
               one context (one sweep launch per step), weighted averages
               over the 1024 runs of each L in FP64 inside the timed region
               (with cpu_baseline_many_runs: independent single-threaded
               oracle processes, one per host core, on runs of this batch);
  serving      500 EA +-J requests arriving at Poisson rate 20/s, L uniform
               in {16, 24, 32, 48, 64}, R = 50000, beta 0 -> 3 in 201
               points, theta = 10, served by continuous batching with
               admission by device-memory footprint: p50/p99 latency and
               flips/ns.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue rate of gfx950: 256 CUs x 4 SIMDs x 16 lanes per clock at
# 2.4 GHz = one 32-bit lane-operation per lane-slot.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Algorithmic 32-bit VALU operations of the bit-sliced Metropolis update
# (each 64-bit word operation counts as two):
# one Philox4x32-10 call = 10 rounds x (2 v_mad_u64_u32 + 2 three-input XORs)
# = 40, plus two bit planes of the most-significant-first comparison
# (select, win, tie, or: 4 per 32-bit half) = 16, so 56 per call; one site
# update of a 64-replica word (four neighbour XORs, the two bond-count
# classes, the flip and the undecided mask) = 28.
OPS_PER_CALL = 56
OPS_PER_WORD = 28
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


LOAD_MS = 25.0   # device work between a host restore and a timed block


def hold_load(ms=LOAD_MS):
    """Keep the device busy for about `ms` milliseconds without touching any
    context (the Philox calibration kernel, about 5 ms per 4096 calls per
    chain).  A restore copies the workspace from host memory while the
    compute units sit idle, and a sweep launched straight after such a gap
    runs several per cent slower for the first ten or so steps; this puts
    each timed block under the load an uninterrupted run is under."""
    import paper_2207_05535_amd as pa
    pa.pa_calibrate_philox(max(1, int(4096 * ms / 5.0)))


def ensure_built():
    import paper_2207_05535_amd as pa
    if not os.path.exists(pa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def kernel_source_hash():
    """Hash of the device sources the HBM counters were taken on, with
    comments and layout removed (an edit of a comment keeps the counters)."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "metropolis.hpp", "philox.hpp", "pa_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2207_05535_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, launches_units):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


TUNING_CACHE = os.path.join(ROOT, "paper_2207_05535_amd", "tuning_cache.json")
# shapes tuned on the two-population +-J workload (L = 32 shared with the FM runs of the batch otherwise)
TWO_POP_TUNING_CACHE = os.path.join(ROOT, "paper_2207_05535_amd", "tuning_cache_two_pop.json")
# shapes tuned on a context like the serving stream (+-J, L in {16,24,32,48,64}, R = 5e4)
SERVING_TUNING_CACHE = os.path.join(ROOT, "paper_2207_05535_amd", "tuning_cache_serving.json")


SEARCH_OUT = [os.path.join(os.getcwd(), "tuning_cache_search.json")]


def tune(ctx, mode, cache=None):
    """Applies autotuned launch shapes: from the committed cache if it holds
    every L of the context, else by a search on the context's own next
    steps (its state is left unchanged).  mode "search" searches afresh and
    merges the result into the file named by --tune-out."""
    if mode == "off":
        return None
    if mode == "search":
        d = os.path.dirname(SEARCH_OUT[0])
        if d:
            os.makedirs(d, exist_ok=True)
        return ctx.autotune(steps=3, cache_path=SEARCH_OUT[0])
    return ctx.autotune(steps=3, cache_path=cache or TUNING_CACHE)


def spread_steps(K, steps, block=5):
    """`steps` temperature steps in blocks of `block` consecutive steps,
    the blocks spread evenly over the whole schedule 1 .. K-1 (the first
    block starts at 1, the last ends at K-1); all steps when
    steps >= K - 1.  Returned as a list of blocks."""
    if steps >= K - 1:
        return [list(range(1, K))]
    nb = max(1, -(-steps // block))
    sizes = [steps // nb + (1 if b < steps % nb else 0) for b in range(nb)]
    last_start = K - sizes[-1]
    starts = [1 + round(b * (last_start - 1) / (nb - 1)) if nb > 1 else 1 for b in range(nb)]
    return [list(range(st, st + sz)) for st, sz in zip(starts, sizes)]


def time_batched(descs, steps, warmup, tune_mode, M=None, per_kernel=True, blocks=None, cache=None):
    """Graph-replayed batched path over `steps` temperature steps (plus the
    weighted average over groups of M runs when M is given), timed with HIP
    events and the host clock; then the same steps eagerly with events
    around every sweep launch (records must be identical).

    blocks: the temperature steps to time, as blocks of consecutive steps
    spread over the schedule (None: steps 1 .. steps in one block).  Each
    block is timed from a checkpoint taken in an untimed pass over the whole
    schedule (which is also the warm-up): restore the state before the
    block (untimed), synchronize, replay the block's steps from the step
    graph, synchronize; the timed region is the sum of those intervals, the
    weighted average after the last block included."""
    import numpy as np
    import torch

    import paper_2207_05535_amd as pa

    ctx = pa.Context(descs, "msc")
    tuned = tune(ctx, tune_mode, cache)
    L0 = descs[0]["L"]
    Kr = len(descs[0]["beta"])
    if blocks is None:
        blocks = [list(range(1, 1 + steps))]
    timed = [i for blk in blocks for i in blk]
    ck = ctx.checkpoint()
    before = {}
    if blocks[0][0] == 1:
        before[1] = ck
    # untimed pass (warm-up; instantiates the step graph), keeping the state
    # before each block (host copies of the workspace)
    at = 1
    for blk in blocks:
        if blk[0] > at:
            ctx.run(at, blk[0])
            at = blk[0]
        torch.cuda.synchronize()
        if blk[0] not in before:
            before[blk[0]] = ctx.checkpoint()
    end = min(Kr, max(at + warmup, timed[-1] + 1))
    if end > at:
        ctx.run(at, end)
    torch.cuda.synchronize()
    log(f"batched path: timing {len(timed)} steps of {len(descs)} run(s) in {len(blocks)} block(s)")
    wall = 0.0
    dev = 0.0
    for k, blk in enumerate(blocks):
        ctx.restore(before[blk[0]])
        hold_load()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        ctx.run(blk[0], blk[-1] + 1)
        if k == len(blocks) - 1:
            wavg = ctx.weighted_average(M if M else 1, pa.PA_W_FULL, 0)   # Sec. IV, FP64 on the device
        ev1.record()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        dev += ev0.elapsed_time(ev1) / 1e3
    obs_graph = ctx.obs()
    flips = sum(int(obs_graph[r, p]["R_i"][i]) * descs[r]["theta"] * descs[r]["L"] ** 2
                for r in range(len(descs)) for p in range(obs_graph.shape[1])
                if p == 0 or descs[r]["overlap"] == pa.PA_Q_TWO_POP for i in timed)
    res = dict(wall_s=wall, dev_s=dev, flips=flips, wavg=wavg, timed=timed, blocks=blocks,
               tuning=dict(ctx.tuning(L0), chunks=ctx.sweep_chunks()), tuned=tuned, obs=obs_graph)
    if per_kernel:
        log("batched path: per-kernel timing pass")
        sweep_ms, step_ms = [], []
        words = calls = sweep_flips = 0
        for blk in blocks:
            ctx.restore(before[blk[0]])
            hold_load()
            torch.cuda.synchronize()
            st0 = ctx.stats()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
                    torch.cuda.Event(enable_timing=True)) for _ in blk]
            for k, i in enumerate(blk):
                a, b, c = evs[k]
                a.record()
                ctx.anneal_step(i)
                ctx.resample(i)
                b.record()
                ctx.sweep(i)
                c.record()
                ctx.measure(i)
            done = torch.cuda.Event(enable_timing=True)
            done.record()
            torch.cuda.synchronize()
            for k in range(len(blk)):
                a, b, c = evs[k]
                nxt = evs[k + 1][0] if k + 1 < len(blk) else done
                sweep_ms.append(b.elapsed_time(c))
                step_ms.append(a.elapsed_time(nxt))
            st1 = ctx.stats()
            words += st1["words"] - st0["words"]
            calls += st1["calls"] - st0["calls"]
            sweep_flips += st1["flips"] - st0["flips"]
        got = ctx.obs()
        same = all(np.array_equal(got[:, :, i], obs_graph[:, :, i]) for i in timed)
        assert same, "graph replay differs from eager steps"
        res.update(sweep_ms=sweep_ms, step_ms=step_ms, words=words, calls=calls, sweep_flips=sweep_flips)
    ctx.close()
    return res


def roofline_of(b, steps):
    sweep_avg_s = sum(b["sweep_ms"]) / len(b["sweep_ms"]) / 1e3
    ops_per_launch = (OPS_PER_CALL * b["calls"] + OPS_PER_WORD * b["words"]) / steps
    achieved = ops_per_launch / sweep_avg_s
    return sweep_avg_s, achieved


def run_plain(desc, timed, warmup, obs_ref):
    """The plain path (int8, one colour of one run per launch, host-driven
    steps) on the same temperature steps as the batched path: each timed
    step from a checkpoint of an untimed pass (consecutive steps in one
    interval); its records must equal the batched path's bit for bit."""
    import numpy as np
    import torch

    import paper_2207_05535_amd as pa
    log("plain path: create")
    pctx = pa.Context([desc], "int8")
    # untimed pass: warm-up, and the state before each run of consecutive timed steps
    segs = []
    for i in timed:
        if segs and segs[-1][-1] == i - 1:
            segs[-1].append(i)
        else:
            segs.append([i])
    before = {}
    pck = pctx.checkpoint()
    at = 1
    for seg in segs:
        while at < seg[0]:
            pctx.step(at)
            at += 1
        torch.cuda.synchronize()
        before[seg[0]] = pctx.checkpoint()
    for i in range(at, 1 + max(warmup, 1)):
        pctx.step(i)
    torch.cuda.synchronize()
    pctx.restore(pck)
    del pck
    torch.cuda.synchronize()
    log(f"plain path: timing {len(timed)} steps")
    sw = []
    wall = dev = 0.0
    calls = words = 0
    last = timed[-1]
    for seg in segs:
        pctx.restore(before[seg[0]])
        hold_load()
        sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in seg]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        st0 = pctx.stats()
        t0 = time.perf_counter()
        e0.record()
        for k, i in enumerate(seg):
            pctx.anneal_step(i)
            pctx.resample(i)
            sev[k][0].record()
            pctx.sweep(i)
            sev[k][1].record()
            pctx.measure(i)
        if seg[-1] == last:
            pw = pctx.weighted_average(1, pa.PA_W_FULL, 0)
        e1.record()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        dev += e0.elapsed_time(e1) / 1e3
        st1 = pctx.stats()
        calls += st1["calls"] - st0["calls"]
        words += st1["words"] - st0["words"]
        for a, b in sev:
            sw.append(a.elapsed_time(b))
    obs_plain = pctx.obs()[0, 0].copy()
    ints = [f for f in pa.PA_OBS_DTYPE.names if f not in ("lnQ", "A")]
    same = all(np.array_equal(obs_plain[f][timed], obs_ref[f][timed]) for f in ints)
    same_fp = bool(np.allclose(obs_plain["A"][timed], obs_ref["A"][timed], rtol=1e-12, atol=0))
    pctx.close()
    return dict(wall_s=wall, dev_s=dev, sweep_ms=sw, bit_exact=bool(same and same_fp),
                free_energy=float(pw[0]["minus_beta_WF"][last]), calls=calls, words=words)


def workload_summary(b, steps, name):
    sweep_avg_s, achieved = roofline_of(b, steps)
    return {
        "workload": name,
        "flips_per_ns": round(b["flips"] / b["wall_s"] / 1e9, 3),
        "flips": b["flips"], "wall_s": round(b["wall_s"], 4), "device_s": round(b["dev_s"], 6),
        "ms_per_step": round(b["wall_s"] * 1e3 / steps, 4),
        "latency_ms_per_step": {"p50": round(percentile(b["step_ms"], 0.5), 4),
                                "p99": round(percentile(b["step_ms"], 0.99), 4)},
        "sweep_kernel": {"name": "k_sweep_msc", "avg_ms": round(sweep_avg_s * 1e3, 4),
                         "flips_per_ns": round(b["sweep_flips"] / steps / sweep_avg_s / 1e9, 3),
                         "alu_frac": round(achieved / PEAK_LANE_OPS, 4),
                         "philox_calls_per_word": round(b["calls"] / max(1, b["words"]), 4)},
        "tuning": b["tuning"],
    }


def run_serving(trace, arena_bytes, max_slots, rate=20.0):
    import paper_2207_05535_amd as pa
    from paper_2207_05535_amd.serve import Server, replay
    srv = Server(arena_bytes, max_slots=max_slots, tuning_cache=SERVING_TUNING_CACHE)
    last = [0.0]

    def progress(done, n, t):
        if t - last[0] >= 5.0 or done == n:
            last[0] = t
            log(f"serving: {done}/{n} requests done at t = {t:.1f} s, {srv.info()['resident']} resident")

    rec, summary = replay(srv, trace, time_scale=20.0 / rate, progress=progress)
    srv.close()
    ok = all(int(r["obs"]["status"].max()) == pa.PA_OK for r in rec)
    emp_rate = len(trace) / (trace[-1][0] * 20.0 / rate)
    mean_flips = summary["flips"] / len(trace)
    offered = emp_rate * mean_flips / 1e9
    cap = summary["busy_flips_per_ns"]
    return {
        "workload": f"EA +-J requests at Poisson rate {rate:g}/s (500 arrivals, trace seed 0xA110000), "
                    "L uniform in {16,24,32,48,64}, R=50000, beta 0->3 in 201 points, theta=10, "
                    "index-shift overlaps; continuous batching, admission by device-memory footprint",
        "requests": len(trace), "arrival_rate_per_s": round(emp_rate, 3), "max_slots": max_slots,
        "arena_GiB": round(arena_bytes / 2**30, 2),
        "p50_latency_s": round(summary["p50_s"], 4), "p99_latency_s": round(summary["p99_s"], 4),
        "mean_latency_s": round(summary["mean_s"], 4), "max_latency_s": round(summary["max_s"], 4),
        "flips_per_ns": round(summary["flips_per_ns"], 3),
        "busy_flips_per_ns": round(cap, 3) if cap else None,
        "offered_flips_per_ns": round(offered, 3),
        "utilisation": round(offered / cap, 3) if cap else None,
        "span_s": round(summary["span_s"], 3), "peak_resident": summary["peak_resident"],
        "all_status_ok": ok,
    }


def run_q_estimators(M=16, K=61):
    """Overlap estimators of Sec. III D side by side on one synthetic +-J
    sample (L=32, R=2e4, theta=10, beta 0->2.4): M runs per estimator in one
    context; per step the whole-step and measurement times (the pairing
    kernels run inside the measurement), and at the last temperature the
    share of runs left out for a family above R_i/2 (Table I) and the
    weighted |q| and q^2 with those runs excluded."""
    import torch

    import paper_2207_05535_amd as pa
    import workloads as W

    out = {"workload": f"{M} runs of EA +-J L=32 on one disorder sample per estimator, R=20000, "
                       f"beta 0->2.4 in {K} points, theta=10, multinomial"}
    for name, ov in (("index_shift", W.Q_INDEX_SHIFT), ("two_populations", W.Q_TWO_POP),
                     ("permutation", W.Q_WANG), ("permutation_random_search", W.Q_WANG_RDM)):
        runs = W.q_comparison_runs(M, overlap=ov, K=K)
        ctx = pa.Context(runs, "msc")
        tune(ctx, "cache")
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K - 1)]
        for k, i in enumerate(range(1, K)):
            a, b, c = evs[k]
            a.record()
            ctx.anneal_step(i)
            ctx.resample(i)
            ctx.sweep(i)
            b.record()
            ctx.measure(i)
            c.record()
        torch.cuda.synchronize()
        step_ms = sum(a.elapsed_time(c) for a, _, c in evs) / (K - 1)
        meas_ms = sum(b.elapsed_time(c) for _, b, c in evs) / (K - 1)
        fs = ctx.family_stats(0)
        wa = ctx.weighted_average(M, pa.PA_W_FULL | pa.PA_W_EXCLUDE_LARGE_FAMILY, 0)[0][K - 1]
        out[name] = {"ms_per_step": round(step_ms, 4), "measure_ms_per_step": round(meas_ms, 4),
                     "excluded_fraction_last": float(fs["excluded"][:, K - 1].mean()),
                     "W_absq_last": float(wa["W_absq"]), "W_q2_last": float(wa["W_q2"]),
                     "runs_included_last": int(M - fs["excluded"][:, K - 1].sum())}
        ctx.close()
        log(f"q estimators: {name} {out[name]}")
    return out


def run_theta_infinity(M=1024, R=20000, L=16, beta_f=0.44, K=89):
    """The theta = infinity limit of Sec. V C (Fig. 9: L = 16 at beta = 0.44)
    beside finite theta: M runs of the L = 16 ferromagnet per theta in one
    context (R = 2e4, beta 0 -> 0.44 in steps of 0.005); the mean, variance
    and skewness of -beta F-hat over the runs at the last temperature, and
    its bias against the exact value from the density of states."""
    import numpy as np

    import paper_2207_05535_amd as pa
    import workloads as W

    N = L * L
    g = pa.pa_exact_dos(L)
    terms = [math.log(gm) - beta_f * (-2 * N + 4 * m) for m, gm in enumerate(g) if gm > 0]
    top = max(terms)
    lnZ = top + math.log(sum(math.exp(t - top) for t in terms))
    out = {"workload": f"{M} runs of the L={L} ferromagnet per theta, R={R}, beta 0->{beta_f} in {K} points, "
                       f"multinomial; -beta F-hat at beta={beta_f}",
           "minus_beta_F_exact": lnZ}
    for name, th in (("theta_inf", W.THETA_EXACT), ("theta_5", 5), ("theta_1", 1)):
        runs = [W.run_desc(L, W.FM, seed=W.RUN_SEED_BASE + 0x300000 + m, R=R, theta=th, K=K, beta_f=beta_f)
                for m in range(M)]
        ctx = pa.Context(runs, "msc")
        tune(ctx, "cache")
        t0 = time.perf_counter()
        ctx.run(1, K)
        A = ctx.obs()[:, 0, K - 1]["A"].astype(np.float64)
        dt = time.perf_counter() - t0
        ctx.close()
        sd = A.std()
        out[name] = {"mean": float(A.mean()), "var": float(A.var()),
                     "skewness": float(((A - A.mean()) ** 3).mean() / sd ** 3) if sd > 0 else 0.0,
                     "bias": float(A.mean() - lnZ), "run_s": round(dt, 3)}
        log(f"theta infinity comparison: {name} {out[name]}")
    return out


def run_bias_vs_M(P=30720, L=10, R=100, K=61, beta_f=0.6, thetas=(1, 5),
                  Ms=(1, 2, 4, 8, 16, 30, 32, 64, 128, 256)):
    """Bias of weighted averages versus M (Sec. V B, Table III, Figs. 2 and
    11) at small synthetic scale: per theta a pool of P runs of the L = 10
    ferromagnet (R = 100, beta 0 -> 0.6 in K points) in one context, weighted
    averages over S = P / M groups for each M on the device; near-critical
    absolute bias (averaged over 0.42 <= beta <= 0.46, relative for c) of
    W[e], W[f] and W_var[c] with bootstrap errors, the exponent b of a fit
    a M^-b, the RMSD at beta = 0.44, var w against Eq. (varWpred) at M = 30,
    and for M = 2 the bias of W[f] beside Wang's (beta/2) var F-hat with the
    fit a + b / beta over beta >= 0.5."""
    import numpy as np

    import paper_2207_05535_amd as pa
    import workloads as W
    from paper_2207_05535_amd import bias as B

    N = L * L
    g = pa.pa_exact_dos(L)
    beta = np.array(W.linear_schedule(beta_f, K))
    ex = [B.exact_fm(g, L, b) for b in beta]
    win = np.where((beta >= 0.42 - 1e-9) & (beta <= 0.46 + 1e-9))[0]
    i44 = int(np.argmin(np.abs(beta - 0.44)))
    out = {"workload": f"pool of {P} runs of the L={L} ferromagnet per theta, R={R}, beta 0->{beta_f} in {K} points, "
                       f"multinomial; exact references from the density of states"}
    for th in thetas:
        runs = [W.run_desc(L, W.FM, seed=W.RUN_SEED_BASE + 0x400000 + 0x10000 * th + m, R=R, theta=th, K=K,
                           beta_f=beta_f) for m in range(P)]
        ctx = pa.Context(runs, "msc")
        tune(ctx, "cache")
        ctx.run(1, K)
        res = {"M": list(Ms)}
        per_obs = {"e": [], "f": [], "c": []}
        errs = {"e": [], "f": [], "c": []}
        rm = []
        for M in Ms:
            w = ctx.weighted_average(M, pa.PA_W_FULL, 0)          # [S, K]
            est = {"e": w["W_e"], "c": w["Wvar_c"], "f": B.weighted_f(w, np.where(beta > 0, beta, np.nan), N)}
            for o in per_obs:
                ref = np.array([x[o] for x in ex])
                dev = est[o][:, win] - ref[win]
                if o == "c":
                    dev = dev / ref[win]

                def near_critical(x, axis=0):
                    return np.abs(x.mean(axis=axis)).mean(axis=-1)
                val, err = B.bootstrap(dev, stat=near_critical, n_boot=400, seed=M)
                per_obs[o].append(float(val))
                errs[o].append(float(err))
            e44 = w["W_e"][:, i44]
            rm.append(float(B.rmsd(e44.mean() - ex[i44]["e"], e44.var())))
            if M == 30:
                res["var_w_M30"] = {"measured": float(w["var_w"][:, i44].mean()),
                                    "predicted": float(w["var_w_pred"][:, i44].mean())}
            if M == 2:
                f2 = est["f"]
                sel = np.where(beta >= 0.5)[0]
                fb = f2[:, sel].mean(axis=0) - np.array([ex[i]["f"] for i in sel])
                wang = B.wang_f_bias(beta[sel], f2[:, sel].var(axis=0), N)
                a, b = B.fit_a_plus_b_over_beta(beta[sel], fb)
                res["f_bias_M2"] = {"beta": [float(x) for x in beta[sel][::2]],
                                    "measured": [float(x) for x in fb[::2]],
                                    "wang_estimate": [float(x) for x in wang[::2]],
                                    "fit_a_plus_b_over_beta": [float(a), float(b)]}
        for o in per_obs:
            y, s = np.array(per_obs[o]), np.array(errs[o])
            res[o] = {"near_critical_abs_bias": [float(x) for x in y], "error": [float(x) for x in s]}
            sig = y > 3 * s          # fit only where the bias stands out of its statistical error
            if sig.sum() >= 3:
                a, b, sb = B.fit_power_law(np.array(Ms, float)[sig], y[sig], s[sig])
                res[o].update(fit_b=float(b), fit_sigma_b=float(sb), fit_a=float(a),
                              fit_M=[int(m) for m in np.array(Ms)[sig]])
            else:
                res[o].update(fit_b=None, fit_sigma_b=None, fit_a=None, fit_M=[])
        res["rmsd_e_beta044"] = rm
        ctx.close()
        out[f"theta_{th}"] = res
        log(f"bias vs M: theta={th} b(e)={res['e']['fit_b']} b(f)={res['f']['fit_b']} b(c)={res['c']['fit_b']}")
    return out


def cpu_baseline(desc, sample_every=8):
    """The oracle (single-threaded C, as it stands) on a bounded sample of
    the same workload at its full size: the L = 64 run with all R = 1e5
    replicas is created (untimed), then temperature step 1 is timed --
    reweighting and resampling, and the measurement, over the whole
    population; the theta = 10 sweeps over every `sample_every`-th replica
    group (the oracle sweeps group by group, so the time scales with the
    number of groups) -- and the sweep time is scaled to all groups.
    A whole step at this size takes minutes on one core."""
    import oracle
    run = oracle.OracleRun(desc)
    G = (desc["R"] + 63) // 64
    groups = list(range(0, G, sample_every))
    t0 = time.perf_counter()
    run.anneal_step(1)
    run.resample(1)
    t1 = time.perf_counter()
    run.sweep_groups(1, groups)
    t2 = time.perf_counter()
    run.measure(1)
    t3 = time.perf_counter()
    R1 = int(run.obs()[0, 1]["R_i"])
    flips = R1 * desc["theta"] * desc["L"] ** 2
    t_sweep = (t2 - t1) * G / len(groups)
    t_step = (t1 - t0) + (t3 - t2) + t_sweep
    return dict(value=flips / t_step / 1e9, unit="spin flips/ns", cores=1, host_cores=os.cpu_count(),
                kind="oracle",
                sample=f"L=64 FM at full size (R=100000, N=4096, theta=10), temperature step 1: reweighting "
                       f"and resampling ({t1 - t0:.2f} s) and measurement ({t3 - t2:.2f} s) over the whole "
                       f"population, the sweeps over every {sample_every}th replica group ({len(groups)} of {G}, "
                       f"{t2 - t1:.1f} s) scaled to all groups; {flips} flips in {t_step:.1f} s (scaled)")


def _oracle_steps(job):
    """One oracle run of a workload, whole temperature steps from i = 1 for
    about max_seconds: (attempted flips, seconds, steps done)."""
    desc, max_seconds = job
    import oracle
    run = oracle.OracleRun(desc)
    t0 = time.perf_counter()
    flips = 0
    i = 0
    while time.perf_counter() - t0 < max_seconds and i + 1 < desc["K"]:
        i += 1
        run.step(i)
        flips += int(run.obs()[0, i]["R_i"]) * desc["theta"] * desc["L"] ** 2
    return flips, time.perf_counter() - t0, i


def cpu_baseline_many_runs(max_seconds=10.0):
    """The oracle for the many-runs workload: P independent single-threaded
    oracle processes on the host cores (P = the cores available, at most
    16), each one run of the 4096-run batch (the four lattice sizes in turn)
    for about max_seconds of whole temperature steps; flips of all processes
    over the longest process time.  Processes are started fresh (spawn), so
    none touches the GPU."""
    import multiprocessing as mp
    import workloads as W
    runs = W.batched_fm_uneven()
    P = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1))
    by_L = {}
    for d in runs:
        by_L.setdefault(d["L"], d)
    Ls = sorted(by_L)
    jobs = [(by_L[Ls[p % len(Ls)]], max_seconds) for p in range(P)]
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_oracle_steps, jobs)
    flips = sum(r[0] for r in res)
    secs = max(r[1] for r in res)
    steps = [r[2] for r in res]
    return dict(value=flips / secs / 1e9, unit="spin flips/ns", cores=P, host_cores=os.cpu_count(),
                kind="oracle", processes=P,
                sample=f"{P} independent oracle processes, each one run of the 4096-run workload (L cycling "
                       f"over {Ls}, R=2000, theta=10, beta 0->0.6 in 150 points), whole steps (ii)-(v) from "
                       f"i=1 for about {max_seconds:g} s (steps done {min(steps)}..{max(steps)}); "
                       f"{flips} flips in {secs:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=199)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", default="headline,plain,two_pop,batched,serving,q_estimators,theta_inf,bias",
                    help="comma-separated subset of headline,plain,two_pop,batched,serving,q_estimators,"
                         "theta_inf,bias "
                         "(for profiling runs; the headline value is null when it is left out)")
    ap.add_argument("--extra-steps", type=int, default=0,
                    help="temperature steps of the two_pop and batched workloads (0: whole schedule)")
    ap.add_argument("--tune", choices=("cache", "search", "off"), default="cache",
                    help="launch shapes: committed autotuner cache (search for missing L), "
                         "a fresh search, or the built-in defaults")
    ap.add_argument("--tune-out", default=SEARCH_OUT[0],
                    help="JSON file the shapes of --tune search are written to")
    ap.add_argument("--serving-slots", type=int, default=12)
    ap.add_argument("--serving-rate", type=float, default=20.0,
                    help="arrival rate of the serving trace in requests/s (the trace's arrival times "
                         "are scaled from its 20/s draw, so the requests and their order are the same)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    SEARCH_OUT[0] = os.path.abspath(args.tune_out)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs one population-annealing "
              "workload per GPU and uses no collectives; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    desc = W.fm_L64_R100k()
    steps = max(1, min(args.steps, desc["K"] - 1))
    warmup = max(1, min(args.warmup, desc["K"] - 1))
    ensure_built()
    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 268435456-byte device-to-device copies")
        del src, dst

    only = set(args.only.split(","))
    if args.quick:
        only &= {"headline", "plain"}
    line = {}
    if "headline" in only:
        line = headline(desc, steps, warmup, args, only)
    else:
        line = {"metric": "spin flips/ns on 1 MI355X (batched vs plain), % of roofline, p99 latency",
                "value": None, "unit": "spin flips/ns", "n_gpus": 1, "steps": steps, "warmup": warmup}
    xs = lambda K: K - 1 if args.extra_steps <= 0 else min(args.extra_steps, K - 1)   # noqa: E731
    if "two_pop" in only:
        d3 = W.ea_L32_two_pop()
        log("two-population EA: L=32, 2 x 200000 replicas")
        b3 = time_batched([d3], xs(d3["K"]), warmup, args.tune, cache=TWO_POP_TUNING_CACHE)
        line["two_pop_ea"] = workload_summary(
            b3, xs(d3["K"]), "EA +-J L=32, two populations of R=200000 on one disorder sample, "
                             "beta 0->3 in 301 points, theta=10, q and link overlap between populations")
        del b3
    if "batched" in only:
        runs = W.batched_fm_uneven()
        log("batched weighted averaging: 4096 runs, L in {8,16,24,32}")
        b4 = time_batched(runs, xs(runs[0]["K"]), warmup, args.tune, M=1024)
        line["batched_4096"] = workload_summary(
            b4, xs(runs[0]["K"]), "4096 FM runs in one context, L in {8,16,24,32} (1024 each), R=2000, "
                                  "beta 0->0.6 in 150 points, theta=10, FP64 weighted averages over "
                                  "the 1024 runs of each L inside the timed region")
        line["batched_4096"]["free_energy_per_L"] = [
            float(b4["wavg"][g]["minus_beta_WF"][xs(runs[0]["K"])]) for g in range(4)]
        del b4
    if "serving" in only:
        trace = W.serving_trace()
        log(f"serving: {len(trace)} requests")
        line["serving"] = run_serving(trace, 4 << 30, args.serving_slots, args.serving_rate)
    if "q_estimators" in only:
        log("overlap estimators: index shift, two populations, permutation pairing")
        line["q_estimators"] = run_q_estimators()
    if "theta_inf" in only:
        log("theta = infinity versus finite theta: spread of -beta F-hat")
        line["theta_inf"] = run_theta_infinity()
    if "bias" in only:
        log("bias versus M of weighted averages")
        line["bias_vs_M"] = run_bias_vs_M()
    if not args.no_cpu_baseline and "headline" in only:
        log("cpu baseline: oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(desc)
    if not args.no_cpu_baseline and "batched" in only:
        log("cpu baseline for the many-runs workload: oracle processes on the host cores")
        line["cpu_baseline_many_runs"] = cpu_baseline_many_runs()
    print(json.dumps(line), flush=True)


def headline(desc, steps, warmup, args, only):
    log(f"headline: L={desc['L']} R={desc['R']}")
    blocks = spread_steps(desc["K"], steps)
    timed = [i for blk in blocks for i in blk]
    steps = len(timed)
    b = time_batched([desc], steps, warmup, args.tune, blocks=blocks)
    value = b["flips"] / b["wall_s"] / 1e9
    sweep_avg_s, achieved = roofline_of(b, steps)
    traffic = measured_traffic("k_sweep_msc", steps)
    line = {
        "metric": "spin flips/ns on 1 MI355X (batched vs plain), % of roofline, p99 latency",
        "value": round(value, 3),
        "unit": "spin flips/ns",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(b["wall_s"] * 1e3 / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "2D Ising ferromagnet L=64 periodic, R=100000, beta 0->0.6 in 200 points, "
                        "theta=10, multinomial resampling (199 temperature steps)",
            "L": 64, "R": 100000, "theta": 10, "K": 200, "steps_timed": steps,
            "timed_steps": ["%d..%d" % (blk[0], blk[-1]) for blk in blocks],
            "timed_betas": [[round(desc["beta"][blk[0]], 4), round(desc["beta"][blk[-1]], 4)] for blk in blocks],
            "timing": ("each block of consecutive steps replayed from the step graph, starting from a "
                       "checkpoint of an untimed pass over the whole schedule, after %.0f ms of untimed "
                       "device work that keeps the device under load past the restore, synchronised "
                       "before and after; the timed region is the sum of those intervals" % LOAD_MS)
                      if len(blocks) > 1 else "one interval",
            "path": "batched: 64 replicas per u64 word, lattice in LDS for all sweeps, "
                    "graph-replayed steps",
        },
        "flips": b["flips"],
        "device_s": round(b["dev_s"], 6),
        "latency_ms_per_step": {"p50": round(percentile(b["step_ms"], 0.5), 4),
                                "p99": round(percentile(b["step_ms"], 0.99), 4)},
        "sweep_kernel": {"name": "k_sweep_msc", "avg_ms": round(sweep_avg_s * 1e3, 4),
                         "flips_per_ns": round(b["sweep_flips"] / steps / sweep_avg_s / 1e9, 3),
                         "philox_calls_per_word": round(b["calls"] / max(1, b["words"]), 4)},
        "tuning": b["tuning"],
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4),
                     "peak": round(PEAK_LANE_OPS / 1e12, 4), "unit": "Tlane-op/s",
                     "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": traffic},
    }
    # the same ceiling calibrated on the device: Philox calls back to back in
    # registers (40 VALU instructions each), at the clock the chip holds
    import paper_2207_05535_amd as pa
    cal = pa.pa_calibrate_philox(4096)
    line["roofline"]["calibrated_peak"] = round(40.0 * cal / 1e12, 4)
    line["roofline"]["frac_of_calibrated"] = round(achieved / (40.0 * cal), 4)
    line["roofline"]["philox_calls_per_s"] = cal
    if not args.no_plain and "plain" in only:
        p = run_plain(desc, timed, warmup, b["obs"][0, 0])
        N = desc["L"] ** 2
        plain_sweep_avg = sum(p["sweep_ms"]) / len(p["sweep_ms"]) / 1e3 / (2 * desc["theta"])
        # algorithmic bytes per int8 colour launch: 2 bytes per attempted
        # flip (read and write the updated spin), N / 2 sites of R replicas
        bytes_launch = 2.0 * (N // 2) * desc["R"]
        # what any one-colour launch must move at least: every spin byte of
        # the run (the colour and its neighbours), then the updated colour
        floor_launch = 1.5 * N * desc["R"]
        traffic_int8 = measured_traffic("k_sweep_int8", 1)
        line["plain_int8"] = {
            "flips_per_ns": round(b["flips"] / p["wall_s"] / 1e9, 3),
            "ms_per_step": round(p["wall_s"] * 1e3 / steps, 4),
            "sweep_launch_avg_ms": round(plain_sweep_avg * 1e3, 4),
            "sweep_hbm_GBps": round(bytes_launch / plain_sweep_avg / 1e9, 1),
            "sweep_hbm_frac": round(bytes_launch / plain_sweep_avg / 1e9 / HBM_PEAK_GBS, 4),
            "one_colour_floor_GBps": round(floor_launch / plain_sweep_avg / 1e9, 1),
            "traffic": traffic_int8,
            "traffic_GBps": (round(traffic_int8 / plain_sweep_avg / 1e9, 1) if traffic_int8 else None),
            # the same Philox and site-update work as the batched sweep, per
            # colour launch, against the integer-VALU peak
            "sweep_alu_frac": round((OPS_PER_CALL * p["calls"] + OPS_PER_WORD * p["words"])
                                    / (steps * 2 * desc["theta"]) / plain_sweep_avg / PEAK_LANE_OPS, 4),
            "bit_exact_vs_batched": p["bit_exact"],
        }
        line["batched_over_plain"] = round(p["wall_s"] / b["wall_s"], 3)
    return line


if __name__ == "__main__":
    main()
