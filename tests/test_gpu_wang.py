"""GPU parity of the permutation pairing of Wang et al. (Sec. III D).

* Step by step against the oracle on small runs (several replica groups and
  a ragged last group, lattices whose site count is not a multiple of 64,
  both resampling kinds, both spin layouts, with and without the random
  search pattern): every record bit-exact, the pairing itself bit-exact at
  every temperature, and the overlap histograms.
* At the size of the paper's comparison (L = 32 spin glass, R = 2 10^4,
  theta = 10, beta up to 2.4): at sampled temperatures the device's pairing
  equals the oracle's pairing computed from the device's own family labels,
  it is a permutation without incestuous pairs, and the overlap sums equal
  a numpy recomputation from the device's spins; a population with a family
  above R_i / 2 has no pairs.
* Runs with permutation pairing batched with index-shift and two-population
  runs in one context give each run's own oracle records.
"""
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


def large_family(fam):
    return 2 * np.bincount(fam).max() > len(fam)


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("kind", [W.Q_WANG, W.Q_WANG_RDM])
@pytest.mark.parametrize("resampling", [W.NEAREST_INT, W.MULTINOMIAL])
def test_stepwise_parity(repr_, kind, resampling):
    say(f"permutation pairing stepwise {repr_} kind={kind} resampling={resampling}")
    d = W.run_desc(10, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5100 + kind, disorder_seed=W.DISORDER_SEED_BASE + 5,
                   R=700, theta=3, K=14, beta_f=2.0, resampling=resampling, overlap=kind, qhist=1)
    orc = oracle.OracleRun(d)
    ctx = pa.Context([d], repr_)
    paired = omitted = 0
    for i in range(d["K"]):
        if i:
            orc.step(i)
            ctx.step(i)
        assert_obs_equal(ctx.obs()[0, 0, i], orc.obs()[0, i], f"i={i}")
        st_o, p_o = orc.pairing(0)
        st_g, p_g = ctx.pairing(0)
        assert st_g == st_o, f"i={i}: status {st_g} != {st_o}"
        if st_o == 0:
            assert np.array_equal(p_g, p_o), f"i={i}: pairing differs"
            paired += 1
        else:
            omitted += 1
    assert np.array_equal(ctx.qhist(0), orc.qhist())
    assert paired >= 5, (paired, omitted)
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("kind", [W.Q_WANG, W.Q_WANG_RDM])
def test_large_families_leave_no_pairs(repr_, kind):
    """A strongly resampled run whose families soon exceed R_i / 2: the
    temperatures without a valid pairing have no pairs, as in the oracle."""
    say(f"permutation pairing with large families {repr_} kind={kind}")
    d = W.run_desc(8, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x3300, disorder_seed=W.DISORDER_SEED_BASE + 3,
                   R=300, R_cap=600, theta=1, K=14, beta_f=2.5, resampling=W.NEAREST_INT, overlap=kind, qhist=1)
    orc = oracle.OracleRun(d).run_all()
    ctx = pa.Context([d], repr_)
    ctx.run(1, d["K"])
    got = ctx.obs()[0, 0]
    assert_obs_equal(got, orc.obs()[0], "all records")
    assert np.array_equal(ctx.qhist(0), orc.qhist())
    assert (got["nPairs"] == 0).sum() >= 5 and (got["nPairs"] > 0).sum() >= 2
    st, _ = ctx.pairing(0)
    assert st == (1 if got["nPairs"][-1] == 0 else 0)
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("kind", [W.Q_WANG, W.Q_WANG_RDM])
@pytest.mark.parametrize("R", [20000, 24000])
def test_full_size_spin_glass_pairing(repr_, kind, R):
    """L = 32 +-J, R = 2 10^4 (the repair's labels fit in LDS) and 2.4 10^4
    (they do not: the repair runs in global memory), theta = 10, beta 0 ->
    2.4 in 61 steps; every fourth temperature is checked."""
    L = 32
    N = L * L
    d = W.run_desc(L, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5200 + kind, disorder_seed=W.DISORDER_SEED_BASE + 32,
                   R=R, theta=10, K=61, beta_f=2.4, resampling=W.MULTINOMIAL, overlap=kind, qhist=1)
    say(f"full-size permutation pairing {repr_} kind={kind}")
    ctx = pa.Context([d], repr_)
    paired = 0
    for i in range(d["K"]):
        if i:
            ctx.step(i)
        if i % 4:
            continue
        s, _, fam, _ = ctx.state(0, 0)
        Ri = len(fam)
        o = ctx.obs()[0, 0, i]
        st, pairs = ctx.pairing(0)
        if large_family(fam):
            assert st == 1 and o["nPairs"] == 0, f"i={i}"
            continue
        assert st == 0 and o["nPairs"] == Ri, f"i={i}"
        pi = oracle.random_permutation(d["seed"], i, 0, Ri, 0)
        sigma = oracle.random_permutation(d["seed"], i, 0, Ri, 1) if kind == W.Q_WANG_RDM else None
        st_o, want = oracle.wang_repair(fam, pi, sigma)
        assert st_o == 0 and np.array_equal(pairs, want), f"i={i}: pairing differs from the oracle's"
        assert np.array_equal(np.sort(pairs), np.arange(Ri)) and np.all(fam[pairs] != fam), f"i={i}"
        a = s.astype(np.int32)
        Q = np.einsum("kn,kn->k", a, a[pairs]).astype(np.int64)
        ab = (a * a[pairs]).reshape(Ri, L, L)
        Ql = ((ab * np.roll(ab, -1, axis=2)).sum(axis=(1, 2)) +
              (ab * np.roll(ab, -1, axis=1)).sum(axis=(1, 2))).astype(np.int64)
        assert o["sumQ"] == Q.sum() and o["sumAbsQ"] == np.abs(Q).sum() and o["sumQ2"] == (Q * Q).sum(), f"i={i}"
        assert o["sumQl"] == Ql.sum() and o["sumQl2"] == (Ql * Ql).sum(), f"i={i}"
        h = ctx.qhist(0)[0, i]
        assert np.array_equal(h, np.bincount((N - Q) // 2, minlength=N + 1)), f"i={i}"
        paired += 1
    assert paired >= 4
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
def test_batched_with_other_overlap_kinds(repr_):
    say(f"permutation pairing batched with other overlap kinds {repr_}")
    base = dict(theta=2, K=9, beta_f=2.0, qhist=1)
    runs = [W.run_desc(8, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5300, disorder_seed=7, R=300, overlap=W.Q_WANG, **base),
            W.run_desc(12, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5301, disorder_seed=8, R=200,
                       overlap=W.Q_INDEX_SHIFT, resampling=W.NEAREST_INT, **base),
            W.run_desc(6, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5302, disorder_seed=9, R=150,
                       overlap=W.Q_WANG_RDM, resampling=W.NEAREST_INT, **base),
            W.run_desc(8, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5303, disorder_seed=10, R=100, overlap=W.Q_TWO_POP,
                       **base)]
    ctx = pa.Context(runs, repr_)
    ctx.run(1, base["K"])
    got = ctx.obs()
    for r, d in enumerate(runs):
        orc = oracle.OracleRun(d).run_all()
        for p in range(orc.npop):
            assert_obs_equal(got[r, p], orc.obs()[p], f"run {r} pop {p}")
        assert np.array_equal(ctx.qhist(r), orc.qhist()), f"run {r}"
    ctx.close()


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("L,R,theta,kind", [(4, 1, 1, W.Q_WANG), (4, 2, 1, W.Q_WANG_RDM), (6, 64, 2, W.Q_WANG),
                                            (4, 65, 1, W.Q_WANG_RDM), (10, 129, 0, W.Q_WANG)])
def test_edge_sizes(repr_, L, R, theta, kind):
    """One replica (never a valid pairing), two replicas, exactly one and
    just over one replica group, and theta = 0, against the oracle."""
    say(f"permutation pairing edge sizes {repr_} L={L} R={R} theta={theta} kind={kind}")
    d = W.run_desc(L, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x5400 + R, disorder_seed=11, R=R, theta=theta, K=6,
                   beta_f=1.0, resampling=W.NEAREST_INT, overlap=kind, qhist=1)
    orc = oracle.OracleRun(d)
    ctx = pa.Context([d], repr_)
    for i in range(d["K"]):
        if i:
            orc.step(i)
            ctx.step(i)
        assert_obs_equal(ctx.obs()[0, 0, i], orc.obs()[0, i], f"i={i}")
        st_o, p_o = orc.pairing(0)
        st_g, p_g = ctx.pairing(0)
        assert st_g == st_o and (st_o != 0 or np.array_equal(p_g, p_o)), f"i={i}"
    if R == 1:
        assert (ctx.obs()[0, 0]["nPairs"] == 0).all()
    assert np.array_equal(ctx.qhist(0), orc.qhist())
    ctx.close()

