"""GPU parity: the HIP path through the C ABI versus the CPU oracle.

Bit-exact: spins, energies, family labels, descendant counts, population
sizes, every integer sum, overlap histograms.  FP64 (ln Q, A and every
weighted average): relative 1e-10 with an absolute floor of 1e-12, the
tolerance the method's FP64 steps are held to (summation order and the
device's log/exp may differ from the oracle's in the last few ulps).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_05535_amd as pa  # noqa: E402

RTOL, ATOL = 1e-10, 1e-12
INT_FIELDS = ["R_i", "sumE", "sumE2", "sumAbsM", "sumM2", "nPairs", "sumQ", "sumAbsQ", "sumQ2",
              "sumQl", "sumQl2", "famSumSq", "famMax", "nFam", "Emin", "status"]
REPRS = ["int8", "msc"]


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def close(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.all(np.abs(a - b) <= RTOL * np.maximum(np.abs(a), np.abs(b)) + ATOL)


def assert_obs_equal(g, o, where=""):
    for f in INT_FIELDS:
        assert np.array_equal(np.asarray(g[f]), np.asarray(o[f])), f"{where}: field {f}: {g[f]} != {o[f]}"
    for f in ("lnQ", "A"):
        assert close(g[f], o[f]), f"{where}: field {f}: {g[f]} vs {o[f]}"


def assert_state_equal(ctx, orc, run, where=""):
    for p in range(orc.npop):
        so, Eo, fo, sto = orc.state(p)
        sg, Eg, fg, rg = ctx.state(run, p)
        if sto != 0:
            continue
        assert sg.shape == so.shape, f"{where} pop {p}: R_i {sg.shape[0]} != {so.shape[0]}"
        assert np.array_equal(sg, so), f"{where} pop {p}: spins differ"
        assert np.array_equal(Eg, Eo), f"{where} pop {p}: energies differ"
        assert np.array_equal(fg, fo), f"{where} pop {p}: families differ"
        ro, _, _ = orc.counts(p)
        assert np.array_equal(rg, ro), f"{where} pop {p}: resampling counts differ"


def stepwise_parity(desc, repr_, state_every=1, qhist=False):
    say(f"stepwise parity {repr_}: L={desc['L']} R={desc['R']} K={desc['K']} model={desc['model']} "
        f"res={desc['resampling']} ov={desc['overlap']}")
    orc = oracle.OracleRun(desc)
    ctx = pa.Context([desc], repr_)
    assert_obs_equal(ctx.obs()[0, :, 0], orc.obs()[:, 0], "i=0")
    assert_state_equal(ctx, orc, 0, "i=0")
    for i in range(1, desc["K"]):
        orc.step(i)
        g = ctx.step(i, read=True)
        assert_obs_equal(g[0], orc.obs()[:, i], f"i={i}")
        if state_every and (i % state_every == 0 or i == desc["K"] - 1):
            assert_state_equal(ctx, orc, 0, f"i={i}")
    assert_obs_equal(ctx.obs()[0], orc.obs(), "all records")
    if qhist:
        assert np.array_equal(ctx.qhist(0), orc.qhist())
    ctx.close()


# ------------------------------------------------------------ small, whole


@pytest.mark.parametrize("repr_", REPRS)
def test_fm_L8_R1000_full_schedule(repr_):
    """Ferromagnet L=8, R=1000, beta 0->1 in 101 points, theta=10,
    multinomial: every record and the full population at every step."""
    stepwise_parity(W.fm_L8_R1000(), repr_)


@pytest.mark.parametrize("repr_", REPRS)
def test_fm_nearest_integer(repr_):
    stepwise_parity(W.fm_L8_R1000(m=3, resampling=W.NEAREST_INT), repr_, state_every=5)


@pytest.mark.parametrize("repr_", REPRS)
def test_ea_two_populations_with_histograms(repr_):
    d = W.run_desc(16, W.EA_PMJ, seed=77, disorder_seed=5, R=700, theta=3, K=31, beta_f=3.0,
                   resampling=W.NEAREST_INT, overlap=W.Q_TWO_POP, qhist=1)
    stepwise_parity(d, repr_, state_every=3, qhist=True)


@pytest.mark.parametrize("repr_", REPRS)
def test_ea_index_shift_ragged(repr_):
    d = W.run_desc(12, W.EA_PMJ, seed=99, disorder_seed=8, R=333, theta=2, K=26, beta_f=2.0,
                   overlap=W.Q_INDEX_SHIFT, qhist=1)
    stepwise_parity(d, repr_, state_every=2, qhist=True)


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("L,R,theta", [(4, 1, 3), (4, 63, 1), (6, 64, 2), (10, 65, 1), (4, 130, 0)])
def test_edge_sizes(repr_, L, R, theta):
    """Smallest lattice, single replica, group-boundary population sizes,
    theta = 0 (no equilibration)."""
    d = W.run_desc(L, W.FM, seed=1234 + R, R=R, theta=theta, K=12, beta_f=1.5,
                   resampling=W.NEAREST_INT if R % 2 else W.MULTINOMIAL,
                   overlap=W.Q_INDEX_SHIFT)
    stepwise_parity(d, repr_)


@pytest.mark.parametrize("repr_", REPRS)
def test_capacity_overflow_freezes(repr_):
    d = W.run_desc(4, W.FM, seed=1, R=64, R_cap=64, theta=0, K=20, beta_f=8.0,
                   resampling=W.NEAREST_INT)
    stepwise_parity(d, repr_)


# -------------------------------------------------- batches, graphs, state


def batch_runs():
    return [
        W.run_desc(8, W.FM, seed=11, R=200, theta=2, K=16, beta_f=0.6),
        W.run_desc(16, W.FM, seed=12, R=130, theta=2, K=16, beta_f=0.6, resampling=W.NEAREST_INT),
        W.run_desc(24, W.FM, seed=13, R=70, theta=1, K=16, beta_f=0.6, overlap=W.Q_INDEX_SHIFT),
        W.run_desc(32, W.EA_PMJ, seed=14, disorder_seed=3, R=64, theta=1, K=16, beta_f=0.6,
                   overlap=W.Q_TWO_POP),
    ]


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_uneven_runs(repr_, graph):
    """Runs of different L, model, resampling and pairing in one context
    (one launch per kernel for all of them) equal the oracle run alone;
    with graph=True the K-1 steps are replays of one captured step graph."""
    runs = batch_runs()
    say(f"batch {repr_} graph={graph}")
    ctx = pa.Context(runs, repr_)
    if graph:
        ctx.run(1, 16)
    else:
        for i in range(1, 16):
            ctx.step(i)
    obs = ctx.obs()
    for r, d in enumerate(runs):
        orc = oracle.OracleRun(d).run_all()
        npop = orc.npop
        assert_obs_equal(obs[r, :npop], orc.obs(), f"run {r}")
        if npop == 1 and ctx.npop == 2:
            assert (obs[r, 1]["R_i"] == 0).all()
        assert_state_equal(ctx, orc, r, f"run {r} final")
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_graph_replays_interleaved_with_eager(repr_):
    """Graph replays mixed with eager steps and host synchronisation give
    the same records as the oracle at every step."""
    d = W.run_desc(8, W.EA_PMJ, seed=5, disorder_seed=2, R=300, theta=2, K=13, beta_f=2.0,
                   resampling=W.NEAREST_INT, overlap=W.Q_INDEX_SHIFT)
    ctx = pa.Context([d], repr_)
    ctx.run(1, 3)
    torch.cuda.synchronize()
    ctx.step(3)
    ctx.run(4, 8)
    ctx.step(8, read=True)
    ctx.run(9, 13)
    orc = oracle.OracleRun(d).run_all()
    assert_obs_equal(ctx.obs()[0], orc.obs(), "records")
    assert_state_equal(ctx, orc, 0, "final")
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_state_between_resampling_and_sweeps(repr_):
    """The resampled population, read between resampling and the sweeps,
    equals the oracle's (labels, spins, copy counts), and the step then
    continues exactly."""
    say(f"state after resampling {repr_}")
    d = W.run_desc(8, W.EA_PMJ, seed=21, disorder_seed=3, R=400, theta=2, K=8, beta_f=1.5,
                   resampling=W.NEAREST_INT, overlap=W.Q_NONE)
    orc = oracle.OracleRun(d)
    ctx = pa.Context([d], repr_)
    for i in range(1, d["K"]):
        orc.anneal_step(i)
        orc.resample(i)
        ctx.anneal_step(i)
        ctx.resample(i)
        so, _, fo, _ = orc.state(0)
        sg, _, fg, rg = ctx.state(0, 0)
        assert np.array_equal(sg, so) and np.array_equal(fg, fo), f"i={i}"
        assert np.array_equal(rg, orc.counts(0)[0]), f"i={i}"
        orc.sweep(i)
        orc.measure(i)
        ctx.sweep(i)
        ctx.measure(i)
        assert_obs_equal(ctx.obs()[0, 0, i], orc.obs()[0, i], f"i={i}")
    assert_state_equal(ctx, orc, 0, "final")
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_checkpoint_restore_bit_exact(repr_):
    d = W.run_desc(8, W.FM, seed=8, R=500, theta=3, K=21, beta_f=1.0, resampling=W.NEAREST_INT,
                   overlap=W.Q_INDEX_SHIFT)
    ctx = pa.Context([d], repr_)
    for i in range(1, 9):
        ctx.step(i)
    ck = ctx.checkpoint()
    for i in range(9, 21):
        ctx.step(i)
    first = ctx.obs().copy()
    s1 = ctx.state(0, 0)
    ctx.restore(ck)
    for i in range(9, 21):
        ctx.step(i)
    second = ctx.obs()
    s2 = ctx.state(0, 0)
    assert first.tobytes() == second.tobytes()
    for a, b in zip(s1, s2):
        assert np.array_equal(a, b)
    # and into a fresh context with another workspace
    ctx2 = pa.Context([d], repr_)
    ctx2.restore(ck)
    for i in range(9, 21):
        ctx2.step(i)
    assert ctx2.obs().tobytes() == first.tobytes()
    # a context of other runs with the same workspace size refuses it
    for other in (W.with_(d, seed=9), W.with_(d, theta=4), W.with_(d, beta_f=0.9)):
        ctx3 = pa.Context([other], repr_)
        with pytest.raises(pa.PAError) as e:
            ctx3.restore(ck)
        assert e.value.status == pa.PA_ERR_ARG
        ctx3.close()
    ctx.close()
    ctx2.close()


def test_restore_after_launch_shape_change():
    """A restore after the launch shapes changed continues with the current
    shapes: the sweep's device work list is the current plan's, not the one
    saved with the checkpoint (items of four replica groups launched with the
    LDS of one would not fit).  The continued run equals the uninterrupted
    one bit for bit, and no sweep item was skipped (the work counters read
    without error)."""
    d = W.run_desc(32, W.FM, seed=0x532, R=20000, theta=2, K=9, beta_f=0.5)
    ref = pa.Context([d], "msc")
    ref.run(1, 9)
    want = (ref.obs().tobytes(), [np.ascontiguousarray(a).tobytes() for a in ref.state(0, 0)], ref.stats())
    ref.close()
    ctx = pa.Context([d], "msc")
    ctx.run(1, 5)
    ck = ctx.checkpoint()
    for threads, groups, dense, persistent, chunks in [(256, 1, 2, 1, 2), (1024, 2, 4, 0, 1)]:
        say(f"restore after shape change: threads={threads} groups={groups} persistent={persistent}")
        ctx.set_tuning(32, threads, groups, dense)
        ctx.set_persistent(persistent)
        ctx.set_sweep_chunks(chunks)
        ctx.restore(ck)
        ctx.run(5, 9)
        got = (ctx.obs().tobytes(), [np.ascontiguousarray(a).tobytes() for a in ctx.state(0, 0)], ctx.stats())
        assert got == want, (threads, groups, persistent)
    ctx.close()


def test_out_of_order_calls_rejected():
    d = W.run_desc(8, W.FM, R=64, theta=1, K=5, beta_f=0.5)
    ctx = pa.Context([d], "msc")
    with pytest.raises(pa.PAError) as e:
        pa.pa_resample(ctx.h, 1)
    assert e.value.status == pa.PA_ERR_STATE
    with pytest.raises(pa.PAError):
        pa.pa_anneal_step(ctx.h, 2)
    ctx.step(1)
    with pytest.raises(pa.PAError):
        pa.pa_run(ctx.h, 3, 4)
    ctx.close()


# ----------------------------------------------------------- weighted average


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("kind", [pa.PA_W_FULL, pa.PA_W_SIMPLE])
def test_weighted_average_parity(repr_, kind):
    """Sec. IV on the device (FP64 log-sum-exp) versus the oracle."""
    M = 8
    runs = [W.run_desc(6, W.EA_PMJ, seed=300 + m, disorder_seed=1, R=150, R_cap=260, theta=2, K=14,
                       beta_f=2.0, resampling=W.NEAREST_INT, overlap=W.Q_INDEX_SHIFT)
            for m in range(2 * M)]
    ctx = pa.Context(runs, repr_)
    ctx.run(1, 14)
    got = ctx.weighted_average(M, kind, 0)
    obs = np.stack([oracle.OracleRun(d).run_all().obs()[0] for d in runs])
    for grp in range(2):
        ref = oracle.weighted_average(obs[grp * M:(grp + 1) * M], runs[0]["beta"], 36, 150, kind)
        assert np.array_equal(got[grp]["n_included"], ref["n_included"])
        for f in pa.PA_WAVG_DTYPE.names:
            if f in ("n_included", "_pad"):
                continue
            assert close(got[grp][f], ref[f]), (grp, f, got[grp][f], ref[f])
    ctx.close()


@pytest.mark.parametrize("M", [1024, 256])
def test_weighted_average_parity_at_benchmark_groupings(M):
    """The device's weighted averages over groups as large as the
    benchmark's (4 groups of 1024 runs; 16 groups of 256), runs of different
    target sizes, half of them nearest-integer (so the full weight's
    R_{k-1}/R factors differ per run), both weight kinds, versus the oracle."""
    n = 4096
    say(f"weighted averages over groups of M={M} ({n} runs)")
    runs = [W.run_desc(8, W.FM, seed=0x3A00 + m, R=40 + 8 * (m % 7), theta=1, K=9, beta_f=0.8,
                       resampling=W.NEAREST_INT if m % 2 else W.MULTINOMIAL) for m in range(n)]
    ctx = pa.Context(runs, "msc")
    ctx.run(1, 9)
    obs_dev = ctx.obs()[:, 0, :]
    obs = np.empty_like(obs_dev)
    for m, d in enumerate(runs):
        obs[m] = oracle.OracleRun(d).run_all().obs()[0]
    for f in INT_FIELDS:
        assert np.array_equal(obs_dev[f], obs[f]), f
    Rs = np.array([d["R"] for d in runs], np.int32)
    for kind in (0, 1):
        got = ctx.weighted_average(M, kind, 0)
        assert got.shape[0] == n // M
        for grp in range(n // M):
            sl = slice(grp * M, (grp + 1) * M)
            ref = oracle.weighted_average(obs[sl], runs[0]["beta"], 64, Rs[sl], kind)
            assert np.array_equal(got[grp]["n_included"], ref["n_included"])
            for f in pa.PA_WAVG_DTYPE.names:
                if f in ("n_included", "_pad"):
                    continue
                assert close(got[grp][f], ref[f]), (kind, grp, f, got[grp][f], ref[f])
    ctx.close()


@pytest.mark.parametrize("overlap", [W.Q_INDEX_SHIFT, W.Q_TWO_POP])
def test_weighted_overlap_distribution_and_family_stats_parity(overlap):
    """Eq. (W_conf_q) on the device, with every weight kind and the
    large-family exclusion (Table I), the exclusion in the overlap averages,
    and the family statistics (Eq. (rho_t)), versus the oracle."""
    say(f"weighted P(q) and family statistics, overlap={overlap}")
    M, L = 6, 6
    N = L * L
    runs = [W.run_desc(L, W.EA_PMJ, seed=500 + m, disorder_seed=4, R=90, theta=1, K=12, beta_f=2.5,
                       overlap=overlap, qhist=1) for m in range(2 * M)]
    ctx = pa.Context(runs, "msc")
    ctx.run(1, 12)
    refs = [oracle.OracleRun(d).run_all() for d in runs]
    npop = 2 if overlap == W.Q_TWO_POP else 1
    obs = [np.stack([r.obs()[p] for r in refs]) for p in range(npop)]
    qh = np.stack([r.qhist()[0] for r in refs])
    other = obs[1] if npop == 2 else None
    seen_large = False
    for kind in (0, 1, 2, 3):
        got_p = ctx.weighted_qhist(M, kind, 0)
        got_a = ctx.weighted_average(M, kind, 0)
        for grp in range(2):
            sl = slice(grp * M, (grp + 1) * M)
            ref_p = oracle.weighted_qhist(obs[0][sl], qh[sl], N, 90, kind=kind,
                                          obs_other=None if other is None else other[sl])
            ref_a = oracle.weighted_average(obs[0][sl], runs[0]["beta"], N, 90, kind=kind,
                                            obs_other=None if other is None else other[sl])
            assert np.array_equal(np.isnan(got_p[grp]), np.isnan(ref_p)), (kind, grp)
            assert close(np.nan_to_num(got_p[grp]), np.nan_to_num(ref_p)), (kind, grp)
            for f in ("W_absq", "W_q2", "W_ql", "W_e", "minus_beta_WF"):
                g, r = got_a[grp][f], ref_a[f]
                assert np.array_equal(np.isnan(g), np.isnan(r)) and close(np.nan_to_num(g), np.nan_to_num(r)), \
                    (kind, grp, f)
    for p in range(npop):
        fs = ctx.family_stats(p)
        for m, r in enumerate(refs):
            ref = oracle.family_stats(r.rho()[p], r.obs()[p], r.obs()[1 - p] if npop == 2 else None)
            for f in ("R_i", "famMax", "large", "excluded"):
                assert np.array_equal(fs[m][f], ref[f]), (p, m, f)
            assert close(fs[m]["rho_t"], ref["rho_t"]), (p, m)
            seen_large |= bool(ref["large"].any())
    assert seen_large, "the runs should reach families above R_i/2"
    ctx.close()


# --------------------------------------------------------- full-size samples


@pytest.mark.parametrize("repr_", REPRS)
def test_full_size_fm_L64_R100k_first_step(repr_):
    """The L=64, R=1e5 ferromagnet at full size: records of temperatures 0
    and 1 (every integer sum, ln Q_1, A_1), all descendant counts, and the
    spins of sampled replica groups after the first theta = 10 sweeps."""
    d = W.fm_L64_R100k()
    groups = [0, 1, 777, (d["R"] - 1) // 64]
    say(f"full size L=64 R=1e5 {repr_}")
    orc = oracle.OracleRun(d)
    orc.anneal_step(1)
    orc.resample(1)
    ro, _, _ = orc.counts(0)
    orc.sweep_groups(1, groups)
    so, Eo, fo, _ = orc.state(0)
    ctx = pa.Context([d], repr_)
    obs0 = ctx.obs()[0, :, 0]
    assert_obs_equal(obs0, orc.obs()[:, 0], "i=0")
    g = ctx.step(1, read=True)[0]
    sg, Eg, fg, rg = ctx.state(0, 0)
    assert np.array_equal(rg, ro)
    assert np.array_equal(fg, fo)
    for gr in groups:
        sl = slice(64 * gr, min(64 * gr + 64, d["R"]))
        assert np.array_equal(sg[sl], so[sl]), f"group {gr}"
        assert np.array_equal(Eg[sl], Eo[sl]), f"group {gr} energies"
    # ln Q_1 and A_1 of step (ii) at full size (the oracle's other sums are
    # not comparable: it swept only the sampled groups)
    orc.measure(1)
    o_ref = orc.obs()[0, 1]
    assert close(g["lnQ"], o_ref["lnQ"]) and close(g["A"], o_ref["A"])
    o1 = g
    # integer sums at full size against the returned configurations
    E = sg.astype(np.int64)
    Ecalc = -(E.reshape(-1, 64, 64) * np.roll(E.reshape(-1, 64, 64), -1, 2)).sum((1, 2)) \
        - (E.reshape(-1, 64, 64) * np.roll(E.reshape(-1, 64, 64), -1, 1)).sum((1, 2))
    assert np.array_equal(Ecalc, Eg)
    M = E.sum(1)
    assert o1["sumE"] == Ecalc.sum() and o1["sumE2"] == (Ecalc * Ecalc).sum()
    assert o1["sumAbsM"] == np.abs(M).sum() and o1["sumM2"] == (M * M).sum()
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_full_size_ea_L32_two_pop_first_step(repr_):
    """EA +-J L=32, two populations of 2e5 on one disorder: records of
    temperature 0 (overlaps of 2e5 pairs) and sampled groups after step 1."""
    d = W.ea_L32_two_pop()
    groups = [0, 1562, 3124]
    say(f"full size EA L=32 2x2e5 {repr_}")
    orc = oracle.OracleRun(d)
    ctx = pa.Context([d], repr_)
    assert_obs_equal(ctx.obs()[0, :, 0], orc.obs()[:, 0], "i=0")
    orc.anneal_step(1)
    orc.resample(1)
    counts = [orc.counts(p)[0] for p in range(2)]
    orc.sweep_groups(1, groups)
    ctx.step(1)
    for p in range(2):
        so, Eo, fo, _ = orc.state(p)
        sg, Eg, fg, rg = ctx.state(0, p)
        assert np.array_equal(rg, counts[p])
        assert np.array_equal(fg, fo)
        for gr in groups:
            sl = slice(64 * gr, 64 * gr + 64)
            assert np.array_equal(sg[sl], so[sl]), f"pop {p} group {gr}"
            assert np.array_equal(Eg[sl], Eo[sl]), f"pop {p} group {gr} energies"
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_full_size_batched_uneven_sampled_runs(repr_):
    """4096 FM runs with L in {8,16,24,32} (1024 each), R=2000, in one
    context; sampled runs (one per L) checked against the oracle over the
    first 4 temperature steps, replayed from the captured step graph."""
    runs = W.batched_fm_uneven()
    say(f"full batch 4096 runs {repr_}")
    ctx = pa.Context(runs, repr_)
    if repr_ == "msc":
        ctx.run(1, 5)
    else:
        for i in range(1, 5):
            ctx.step(i)
    obs = ctx.obs()
    for r in (5, 1024 + 17, 2048 + 1000, 3072 + 1023):
        d = runs[r]
        orc = oracle.OracleRun(d)
        for i in range(1, 5):
            orc.step(i)
        assert_obs_equal(obs[r, 0, :5], orc.obs()[0, :5], f"run {r}")
        assert_state_equal(ctx, orc, r, f"run {r}")
    ctx.close()


# ------------------------------------------------------------- tuning shapes


@pytest.mark.parametrize("threads,groups,dense,pooled", [(64, 1, 0, 0), (256, 2, 3, 0), (1024, 1, 16, 0),
                                                         (128, 3, 1, 0), (512, 5, 2, 0), (64, 1, 0, 1),
                                                         (256, 2, 3, 1), (1024, 2, 1, 1), (512, 1, 4, 1)])
def test_tuning_shapes_do_not_change_results(threads, groups, dense, pooled):
    """Every launch shape of the batched sweep (threads per workgroup, replica
    groups per workgroup, lockstep calls before compaction, per-wavefront or
    pooled lists for the compacted rounds) gives the oracle's results bit for
    bit."""
    say(f"tuning shape threads={threads} groups={groups} dense={dense} pooled={pooled}")
    runs = batch_runs()
    ctx = pa.Context(runs, "msc")
    ctx.set_pooled(pooled)
    for d in runs:
        ctx.set_tuning(d["L"], threads, groups, dense)
    ctx.run(1, 16)
    obs = ctx.obs()
    for r, d in enumerate(runs):
        orc = oracle.OracleRun(d).run_all()
        assert_obs_equal(obs[r, :orc.npop], orc.obs(), f"run {r}")
        assert_state_equal(ctx, orc, r, f"run {r} final")
    ctx.close()


def test_sweep_statistics_are_shape_independent():
    """The sweeps' counters (word-site updates, Philox calls, attempted flips)
    are properties of the runs: a site makes exactly the calls up to the one
    that decides its last undecided replica, whatever the representation,
    launch shape, list scheme or tail.  Attempted flips equal
    sum_i theta N R_i and word-sites sum_i theta N ceil(R_i / 64) over the
    records, at every shape."""
    runs = batch_runs()
    say("sweep statistics across representations and shapes")
    flips = words = 0
    ctx = pa.Context(runs, "int8")
    ctx.run(1, 16)
    obs = ctx.obs()
    for r, d in enumerate(runs):
        for p in range(2 if d["overlap"] == W.Q_TWO_POP else 1):
            Ri = obs[r, p, 1:]["R_i"].astype(np.int64)
            flips += int((d["theta"] * d["L"] ** 2 * Ri).sum())
            words += int((d["theta"] * d["L"] ** 2 * ((Ri + 63) // 64)).sum())
    ref = ctx.stats()
    ctx.close()
    assert ref["flips"] == flips and ref["words"] == words, (ref, flips, words)
    assert ref["calls"] > 0
    for threads, groups, dense, pooled in [(64, 1, 0, 0), (256, 2, 3, 0), (1024, 1, 16, 0), (512, 1, 3, 0),
                                           (64, 1, 0, 1), (1024, 2, 1, 1), (512, 1, 4, 1)]:
        ctx = pa.Context(runs, "msc")
        ctx.set_pooled(pooled)
        for d in runs:
            ctx.set_tuning(d["L"], threads, groups, dense)
        ctx.run(1, 16)
        got = ctx.stats()
        ctx.close()
        assert got == ref, (threads, groups, dense, pooled, got, ref)


def test_mixed_sizes_one_launch_per_size():
    """Runs of two lattice sizes, each size with enough replica groups to
    fill the chip with the launch shapes of the tuning cache, sweep in one
    launch per size with the kernels compiled for each size (the plan reports
    two launches, where a mix of small runs keeps one dispatching launch);
    every run's records, spins, energies and family labels equal those of
    the same run swept in a context of its own size, which the single-size
    tests tie to the oracle."""
    import json
    import os
    cache = os.path.join(os.path.dirname(pa.__file__), "tuning_cache.json")
    with open(cache) as fh:
        shape = {e["L"]: e for e in json.load(fh)["entries"] if e["repr"] == "msc"}
    Ls = (16, 32)
    runs = W.batched_fm_uneven(n_per_L=192, Ls=Ls, R=2000, K=6)

    def context(rs, sizes):
        c = pa.Context(rs, "msc")
        for L in sizes:
            c.set_tuning(L, shape[L]["threads"], shape[L]["groups"], shape[L]["dense"])
        c.set_persistent(0)
        return c

    say("mixed sizes, one sweep launch per size")
    mixed = context(runs, Ls)
    assert mixed.sweep_launches() == 2
    mixed.run(1, 6)
    small = context(runs[:2] + runs[192:194], Ls)
    assert small.sweep_launches() == 1   # too few groups per size to fill the chip
    small.close()
    obs = mixed.obs()
    for k, L in enumerate(Ls):
        part = runs[k * 192:(k + 1) * 192]
        alone = context(part, (L,))
        assert alone.sweep_launches() == 1
        alone.run(1, 6)
        ref = alone.obs()
        assert obs[k * 192:(k + 1) * 192].tobytes() == ref.tobytes(), f"L={L}: records differ"
        for r in (0, 77, 191):
            for a, b in zip(mixed.state(k * 192 + r, 0), alone.state(r, 0)):
                assert np.array_equal(np.asarray(a), np.asarray(b)), f"L={L} run {r}: state differs"
        alone.close()
    mixed.close()


def _digest(ctx, d, steps):
    import hashlib
    h = hashlib.sha256()
    h.update(ctx.obs()[0, :, :1 + steps].tobytes())
    for p in range(2 if d["overlap"] == W.Q_TWO_POP else 1):
        for a in ctx.state(0, p):
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("workload", ["fm_L64_R100k", "ea_L32_two_pop", "fm_L64_R100k_theta1"])
def test_sweep_chunks_bit_exact_at_full_size(workload):
    """Items split into chunks of consecutive sweeps on the persistent grid
    (each chunk waiting on the device for the previous chunk of its replica
    groups) give the records, states and work counters of whole items.  At
    these sizes the items outnumber the resident workgroups (1563 of one
    group at L = 64 with 512 threads; 3125 of two groups at L = 32), so the
    chunks are really used; the automatic choice (0) is checked too.  With
    theta = 1 every chunk but one holds no sweep at all (it only loads and
    stores its lattices)."""
    if workload == "ea_L32_two_pop":
        d = W.ea_L32_two_pop()
    else:
        d = W.fm_L64_R100k()
        if workload.endswith("theta1"):
            d = W.with_(d, theta=1)
    G = 1 if d["L"] == 64 else 2
    steps = 3
    ref = None
    for K in (1, 2, 3, 4, 0):
        say(f"sweep chunks {workload}: K={K}")
        ctx = pa.Context([d], "msc")
        ctx.set_tuning(d["L"], 512, G, 3)
        ctx.set_persistent(1)
        ctx.set_sweep_chunks(K)
        used = ctx.sweep_chunks()
        assert used == K if K else used >= 1, (K, used)
        ctx.run(1, 1 + steps)
        got = (_digest(ctx, d, steps), tuple(int(x) for x in ctx.stats().values()))
        ctx.close()
        if ref is None:
            ref = got
        assert got == ref, (K, used)
    with pytest.raises(pa.PAError):
        ctx = pa.Context([d], "msc")
        try:
            ctx.set_sweep_chunks(5)
        finally:
            ctx.close()


def test_sweep_chunks_whole_schedule():
    """The headline workload over its whole schedule (199 steps, beta up to
    0.6) with the cache's three chunks of sweeps on the persistent grid
    equals the same run with whole items: every record, the final state and
    the work counters."""
    d = W.fm_L64_R100k()
    got = []
    for K in (1, 3):
        say(f"whole schedule with {K} chunk(s)")
        ctx = pa.Context([d], "msc")
        ctx.set_tuning(64, 512, 1, 3)
        ctx.set_persistent(1)
        ctx.set_sweep_chunks(K)
        assert ctx.sweep_chunks() == K
        ctx.run(1, d["K"])
        got.append((_digest(ctx, d, d["K"] - 1), ctx.stats()))
        ctx.close()
    assert got[0] == got[1]


@pytest.mark.parametrize("repr_", REPRS)
def test_multichunk_and_small_runs_in_one_context(repr_):
    """A run of several 2048-replica chunks next to single-chunk runs: the
    multinomial draws of the large run spread over several workgroups per
    chunk while the small runs draw in one, families crossing chunk
    boundaries at low temperature; every record and the final state equal
    the oracle's."""
    runs = [W.run_desc(8, W.FM, seed=W.RUN_SEED_BASE + 0x7100, R=5000, theta=2, K=14, beta_f=1.2),
            W.run_desc(8, W.FM, seed=W.RUN_SEED_BASE + 0x7101, R=300, theta=2, K=14, beta_f=1.2),
            W.run_desc(6, W.FM, seed=W.RUN_SEED_BASE + 0x7102, R=2100, theta=1, K=14, beta_f=1.2,
                       resampling=W.NEAREST_INT)]
    say(f"multi-chunk and small runs {repr_}")
    ctx = pa.Context(runs, repr_)
    ctx.run(1, 14)
    obs = ctx.obs()
    for r, d in enumerate(runs):
        orc = oracle.OracleRun(d).run_all()
        assert_obs_equal(obs[r, :orc.npop], orc.obs(), f"run {r}")
        assert_state_equal(ctx, orc, r, f"run {r} final")
    ctx.close()


@pytest.mark.parametrize("L,model", [(8, W.FM), (16, W.EA_PMJ), (24, W.FM), (24, W.EA_PMJ), (32, W.FM),
                                     (48, W.FM), (48, W.EA_PMJ), (64, W.EA_PMJ)])
@pytest.mark.parametrize("persistent", [0, 1])
def test_single_size_kernel(L, model, persistent):
    """A context whose runs share one lattice size and model launches the
    sweep kernel compiled for that size: one workgroup per item or the
    persistent grid, with two runs of different seeds and population sizes;
    every record and the final states equal the oracle's."""
    say(f"single-size sweep kernel L={L} model={model} persistent={persistent}")
    runs = [W.run_desc(L, model, seed=W.RUN_SEED_BASE + 0x7200 + L, disorder_seed=7, R=300, theta=2, K=10,
                       beta_f=1.0),
            W.run_desc(L, model, seed=W.RUN_SEED_BASE + 0x7300 + L, disorder_seed=7, R=130, theta=3, K=10,
                       beta_f=1.0, resampling=W.NEAREST_INT)]
    ctx = pa.Context(runs, "msc")
    ctx.set_persistent(persistent)
    ctx.run(1, 10)
    obs = ctx.obs()
    for r, d in enumerate(runs):
        orc = oracle.OracleRun(d).run_all()
        assert_obs_equal(obs[r, :orc.npop], orc.obs(), f"run {r}")
        assert_state_equal(ctx, orc, r, f"run {r} final")
    ctx.close()
