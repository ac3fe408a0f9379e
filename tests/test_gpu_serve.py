"""Serving (continuous batching) and autotuner on the GPU.

Serving: every request's records must be the same when it runs in the mix
(admitted as slots and arena space free up, sharing launches with runs at
other temperatures) as when its descriptor runs alone in a context, bit for
bit in every field; one small request is also checked against the oracle.

Autotuner: the tuned shape must leave the records bit-identical to the
untuned run, reject no candidate, and be reproduced from its JSON cache
without a search.
"""
import json
import sys

import numpy as np
import pytest

import oracle
import paper_2207_05535_amd as pa
import workloads as W
from paper_2207_05535_amd.serve import Server, replay

pytestmark = pytest.mark.gpu

INT_FIELDS = [f for f in pa.PA_OBS_DTYPE.names if f not in ("lnQ", "A")]


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def mixed_trace():
    """Twelve requests of several sizes, models, resampling kinds, overlap
    estimators (permutation pairing among them), schedule lengths and one at
    theta = infinity, with staggered arrivals."""
    specs = [
        (8, W.FM, W.MULTINOMIAL, W.Q_NONE, 12, 300),
        (12, W.EA_PMJ, W.NEAREST_INT, W.Q_INDEX_SHIFT, 9, 500),
        (16, W.EA_PMJ, W.MULTINOMIAL, W.Q_TWO_POP, 15, 700),
        (10, W.FM, W.NEAREST_INT, W.Q_INDEX_SHIFT, 7, 129),
        (8, W.EA_PMJ, W.MULTINOMIAL, W.Q_INDEX_SHIFT, 20, 64),
        (16, W.FM, W.MULTINOMIAL, W.Q_NONE, 11, 1000),
        (24, W.EA_PMJ, W.MULTINOMIAL, W.Q_INDEX_SHIFT, 6, 400),
        (6, W.EA_PMJ, W.NEAREST_INT, W.Q_TWO_POP, 13, 250),
        (32, W.FM, W.MULTINOMIAL, W.Q_INDEX_SHIFT, 5, 200),
        (12, W.EA_PMJ, W.MULTINOMIAL, W.Q_WANG_RDM, 10, 300),
        (10, W.FM, W.NEAREST_INT, W.Q_WANG, 8, 260),
        (8, W.FM, W.MULTINOMIAL, W.Q_NONE, 9, 400, W.THETA_EXACT),
    ]
    out = []
    for q, (L, model, rs, ov, K, R, *th) in enumerate(specs):
        d = W.run_desc(L, model, seed=W.RUN_SEED_BASE + 0x7000 + q,
                       disorder_seed=W.DISORDER_SEED_BASE + 0x70 + q, R=R, theta=th[0] if th else 3, K=K,
                       beta_f=1.5 if model == W.EA_PMJ else 0.6, resampling=rs, overlap=ov)
        out.append((0.002 * q, d))
    return out


def alone(desc, repr_):
    ctx = pa.Context([desc], repr_)
    ctx.run(1, desc["K"])
    obs = ctx.obs()[0]          # [n_pop][K]
    ctx.close()
    return np.ascontiguousarray(obs.T)   # [K][n_pop], the server's layout


def assert_same(a, b, what):
    for f in pa.PA_OBS_DTYPE.names:
        assert np.array_equal(a[f], b[f]), (what, f)


@pytest.mark.parametrize("repr_", ["msc", "int8"])
def test_each_request_same_alone_and_in_the_mix(repr_):
    say(f"serving mix vs alone, {repr_}")
    trace = mixed_trace()
    # everything arrives at once and three slots serve it: requests wait and
    # are admitted as earlier ones finish
    srv = Server(64 << 20, max_slots=3, repr_=repr_)
    rec, summary = replay(srv, trace, time_scale=0.0)
    assert summary["peak_resident"] == 3
    for q, (_, d) in enumerate(trace):
        assert rec[q]["admit"] is not None and rec[q]["finish"] >= rec[q]["admit"]
        assert_same(rec[q]["obs"], alone(d, repr_), f"request {q}")
    assert srv.info()["resident"] == 0
    srv.close()


def test_serving_tuned_shapes_on_large_lattices():
    """The launch shapes the serving benchmark loads (1024 threads, four
    lockstep calls, two or three replica groups per workgroup at L = 64, 48)
    on +-J requests of L = 48 and 64 next to smaller ones: each request's
    records in the mix equal those of the same descriptor alone in a
    context with default shapes, and the L = 48 and L = 64 requests equal
    the oracle's."""
    import os
    cache = os.path.join(os.path.dirname(pa.__file__), "tuning_cache_serving.json")
    say("serving mix with the serving tuning cache, L up to 64")
    specs = [(64, 500, 8), (48, 700, 9), (16, 900, 10), (32, 600, 7), (64, 300, 6), (24, 800, 8)]
    trace = []
    for q, (L, R, K) in enumerate(specs):
        d = W.run_desc(L, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x7400 + q, disorder_seed=W.DISORDER_SEED_BASE + 0x740 + q,
                       R=R, theta=3, K=K, beta_f=2.0, overlap=W.Q_INDEX_SHIFT)
        trace.append((0.0, d))
    srv = Server(256 << 20, max_slots=3, repr_="msc", tuning_cache=cache)
    rec, summary = replay(srv, trace, time_scale=0.0)
    srv.close()
    assert summary["peak_resident"] == 3
    for q, (_, d) in enumerate(trace):
        assert_same(rec[q]["obs"], alone(d, "msc"), f"request {q}")
    for q in (0, 1):
        d = trace[q][1]
        o = oracle.OracleRun(d).run_all().obs()
        got = rec[q]["obs"]
        for f in INT_FIELDS:
            assert np.array_equal(got[f][:, 0], o[f][0]), (q, f)
        np.testing.assert_allclose(got["A"][:, 0], o["A"][0], rtol=1e-10, atol=1e-12)


def test_request_in_the_mix_matches_the_oracle():
    say("serving mix vs oracle")
    trace = mixed_trace()
    srv = Server(64 << 20, max_slots=4)
    rec, _ = replay(srv, trace, time_scale=1.0)     # arrivals in real time, 2 ms apart
    srv.close()
    for q in (1, 7):            # nearest-integer with index shift; two populations
        d = trace[q][1]
        ref = oracle.OracleRun(d)
        ref.run_all()
        o = ref.obs()           # [n_pop][K]
        got = rec[q]["obs"]
        for p in range(o.shape[0]):
            for f in INT_FIELDS:
                assert np.array_equal(got[f][:, p], o[f][p]), (q, p, f)
            np.testing.assert_allclose(got["lnQ"][:, p], o["lnQ"][p], rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(got["A"][:, p], o["A"][p], rtol=1e-10, atol=0)


def test_admission_by_footprint_and_reuse():
    say("serving admission by footprint")
    d = W.run_desc(16, W.EA_PMJ, R=2000, theta=2, K=6, beta_f=1.0, overlap=W.Q_INDEX_SHIFT)
    fp = pa.pa_server_footprint(d, "msc")
    # room for two such runs (their tables are shared), not three
    arena = 2 * fp + fp // 2
    srv = Server(arena, max_slots=8)
    descs = [W.with_(d, seed=W.RUN_SEED_BASE + 0x900 + k) for k in range(3)]
    s0 = srv.admit(descs[0])
    s1 = srv.admit(descs[1])
    assert s0 is not None and s1 is not None and s0 != s1
    assert srv.admit(descs[2]) is None          # does not fit now
    assert srv.info()["resident"] == 2
    fin = []
    for _ in range(d["K"] - 1):
        fin += srv.step()
    assert sorted(fin) == sorted([s0, s1])
    o0 = srv.read_obs(s0, descs[0])
    srv.release(s0)
    s2 = srv.admit(descs[2])                     # fits after the release
    assert s2 is not None
    for _ in range(d["K"] - 1):
        srv.step()
    o2 = srv.read_obs(s2, descs[2])
    srv.release(s1)
    srv.release(s2)
    assert srv.info()["bytes_used"] > 0          # the work lists stay allocated
    srv.close()
    assert_same(o0, alone(descs[0], "msc"), "first")
    assert_same(o2, alone(descs[2], "msc"), "reused memory")


def test_autotune_keeps_results_and_uses_cache(tmp_path):
    say("autotune invariance and cache")
    runs = W.batched_fm_uneven(n_per_L=6, Ls=(8, 16, 24, 32), R=300, K=10)
    ref = pa.Context(runs, "msc")
    ref.run(1, 10)
    want = ref.obs()
    ref.close()

    cache = str(tmp_path / "tune.json")
    ctx = pa.Context(runs, "msc")
    ctx.run(1, 3)
    res = ctx.autotune(steps=2, cache_path=cache)
    assert res["tried"] > 10 and res["rejected"] == 0
    shapes = {L: ctx.tuning(L) for L in (8, 16, 24, 32)}
    chunks = ctx.sweep_chunks()
    ctx.run(3, 10)                               # continues exactly as untuned
    assert ctx.obs().tobytes() == want.tobytes()
    ctx.close()

    entries = json.load(open(cache))["entries"]
    assert sorted(e["L"] for e in entries) == [8, 16, 24, 32]

    ctx2 = pa.Context(runs, "msc")
    res2 = ctx2.autotune(steps=2, cache_path=cache)
    assert res2["tried"] == 0
    assert {L: ctx2.tuning(L) for L in (8, 16, 24, 32)} == shapes
    assert ctx2.sweep_chunks() == chunks
    assert all("chunks" in e for e in entries)
    ctx2.run(1, 10)
    assert ctx2.obs().tobytes() == want.tobytes()
    ctx2.close()


def test_persistent_grid_and_pooled_lists_same_results():
    say("persistent sweep grid and pooled list invariance")
    runs = W.batched_fm_uneven(n_per_L=5, Ls=(8, 16, 24, 32), R=500, K=8)
    a = pa.Context(runs, "msc")
    a.run(1, 8)
    b = pa.Context(runs, "msc")
    b.set_persistent(1)
    assert b.tuning(16)["persistent"] == 1
    b.run(1, 4)
    b.set_persistent(0)
    b.set_pooled(1)
    assert b.tuning(16)["pooled"] == 1
    b.run(4, 6)
    b.set_persistent(1)
    for i in range(6, 8):
        b.step(i)
    assert a.obs().tobytes() == b.obs().tobytes()
    assert a.stats() == b.stats()
    a.close()
    b.close()
