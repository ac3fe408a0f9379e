"""pa_create_static: the context in the library's own device array, for
callers that cannot allocate, against pa_create with a caller workspace.

Two contexts in a row on the same array, the second smaller than the first:
every record (bit-exact integers, ln Q and A to the last bit as well, since
both run the same kernels in the same order) and the final state equal those
of the same runs created with pa_create.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_05535_amd as pa  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_both(runs, repr_, graph):
    out = []
    for static in (False, True):
        ctx = pa.Context(runs, repr_, static_workspace=static)
        if graph:
            ctx.run(1, runs[0]["K"])
        else:
            for i in range(1, runs[0]["K"]):
                ctx.step(i)
        obs = ctx.obs()
        states = [ctx.state(r, p) for r in range(len(runs)) for p in range(ctx.npop)
                  if p == 0 or runs[r]["overlap"] == pa.PA_Q_TWO_POP]
        wavg = ctx.weighted_average(len(runs), pa.PA_W_FULL, 0)
        ctx.close()
        out.append((obs, states, wavg))
    return out


@pytest.mark.parametrize("repr_", ["msc", "int8"])
def test_static_workspace_matches_caller_workspace(repr_):
    large = [W.run_desc(16, W.EA_PMJ, seed=0x57A0 + m, disorder_seed=3, R=3000, R_cap=3900, theta=3, K=12,
                        beta_f=1.5, resampling=W.NEAREST_INT, overlap=W.Q_TWO_POP) for m in range(2)]
    small = [W.run_desc(8, W.FM, seed=0x57B0, R=500, theta=2, K=9, beta_f=0.8, overlap=W.Q_INDEX_SHIFT)]
    assert pa.pa_workspace_size(small, repr_) < pa.pa_workspace_size(large, repr_)
    for name, runs, graph in (("large", large, True), ("small", small, False)):
        say(f"static workspace {repr_} {name}")
        (o1, s1, w1), (o2, s2, w2) = run_both(runs, repr_, graph)
        assert o1.tobytes() == o2.tobytes(), name
        assert w1.tobytes() == w2.tobytes(), name
        for a, b in zip(s1, s2):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), name


def test_static_workspace_limits():
    say("static workspace limits")
    d = W.run_desc(8, W.FM, seed=0x57C0, R=200, theta=1, K=4, beta_f=0.5)
    a = pa.Context([d], "msc", static_workspace=True)
    with pytest.raises(pa.PAError) as e:        # the array is held by a live context
        pa.Context([d], "msc", static_workspace=True)
    assert e.value.status == pa.PA_ERR_STATE
    a.close()
    b = pa.Context([d], "msc", static_workspace=True)   # released by pa_destroy
    b.run(1, 4)
    b.close()
    big = W.fm_L64_R100k(R=400_000)                      # about 1.6 GB as int8
    assert pa.pa_workspace_size([big], "int8") > pa.PA_STATIC_WORKSPACE_BYTES
    with pytest.raises(pa.PAError) as e:
        pa.Context([big], "int8", static_workspace=True)
    assert e.value.status == pa.PA_ERR_NOMEM
