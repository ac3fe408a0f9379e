"""Oracle pins for weighted averaging (Sec. IV), CPU only.

Identities of the paper (M = 1, identical runs, Machta's telescoped free
energy for constant R, the W_var >= W lower bound) and its convergence
theorem (bias of configurational weighted averages vanishes as M grows when
no equilibration is done, Sec. IV D) checked against exact enumeration.
"""
import math

import numpy as np
import pytest

import exact
import oracle
import workloads as W


@pytest.fixture(scope="module")
def small_pool():
    d = W.run_desc(4, W.FM, seed=77, R=16, theta=1, K=7, beta_f=0.9)
    return d, oracle.many_runs_obs(d, 64)


def test_single_run_weight_is_one(small_pool):
    """M = 1: w = 1, so W[O] = O and W_var equals the single-run estimator;
    -beta W[F] = A."""
    d, obs = small_pool
    out = oracle.weighted_average(obs[:1], d["beta"], 16, d["R"], kind=0)
    o = obs[0]
    R = o["R_i"].astype(float)
    assert np.allclose(out["W_e"], o["sumE"] / (16 * R), rtol=1e-14, atol=0)
    assert np.allclose(out["minus_beta_WF"], o["A"], rtol=1e-14)
    assert np.allclose(out["Wvar_c"], out["Wconf_c"], rtol=1e-14)
    assert (out["var_w"] == 0).all() and (out["n_included"] == 1).all()


def test_identical_runs_equal_weights(small_pool):
    """M copies of one run: every weight is 1/M, W[O] = O, var w = 0 and
    -beta W[F] = A (weighting on the level of partition functions)."""
    d, obs = small_pool
    rep = np.repeat(obs[:1], 5, axis=0)
    out = oracle.weighted_average(rep, d["beta"], 16, d["R"], kind=1)
    one = oracle.weighted_average(obs[:1], d["beta"], 16, d["R"], kind=1)
    for f in ("W_e", "W_m", "Wconf_c", "Wvar_c", "minus_beta_WF"):
        assert np.allclose(out[f], one[f], rtol=1e-13, atol=1e-13)
    assert np.allclose(out["var_w"], 0.0, atol=1e-30)


def test_machta_identity_constant_population(small_pool):
    """Multinomial resampling with equal R: the incremental weighted free
    energy telescopes to ln[(1/M) sum_m exp(-beta_i F_i^(m))], Eq. (W_F_machta),
    and the full and simplified weights coincide."""
    d, obs = small_pool
    M = obs.shape[0]
    full = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=0)
    simp = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=1)
    A = obs["A"]
    amax = A.max(axis=0)
    machta = amax + np.log(np.exp(A - amax).sum(axis=0) / M)
    assert np.allclose(full["minus_beta_WF"], machta, rtol=1e-12, atol=1e-12)
    for f in ("W_e", "W_m2", "Wvar_c", "Wvar_chi", "minus_beta_WF"):
        assert np.allclose(full[f], simp[f], rtol=1e-13, atol=1e-13)


def test_wvar_lower_bound():
    """W_var[K] = W[K] + sum_m w (O_m - W[O])^2 >= W[K], Eq. (Wvar_bound), for
    the heat capacity and the susceptibility; nearest-integer runs."""
    d = W.run_desc(4, W.FM, seed=5, R=12, R_cap=40, theta=1, K=8, beta_f=1.0,
                   resampling=W.NEAREST_INT)
    obs = oracle.many_runs_obs(d, 40)
    for kind in (0, 1):
        out = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=kind)
        assert (out["Wvar_c"] >= out["Wconf_c"] - 1e-15).all()
        assert (out["Wvar_chi"] >= out["Wconf_chi"] - 1e-15).all()
        assert (out["Wvar_c"][1:] > out["Wconf_c"][1:]).any()


def test_weighted_variance_is_variance_of_weighted_moments():
    """W_var[c] equals beta^2 N (W[e^2] - W[e]^2), Eq. (Wvar_C), where W[e^2]
    averages the per-run population means of (E/N)^2."""
    d = W.run_desc(4, W.EA_PMJ, seed=8, R=10, theta=1, K=6, beta_f=1.4)
    obs = oracle.many_runs_obs(d, 30)
    out = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=1)
    b = np.asarray(d["beta"])
    direct = b ** 2 * 16 * (out["W_e2"] - out["W_e"] ** 2)
    assert np.allclose(out["Wvar_c"], direct, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("model,resampling", [(W.FM, W.MULTINOMIAL), (W.EA_PMJ, W.MULTINOMIAL),
                                               (W.FM, W.NEAREST_INT)])
def test_weighted_average_bias_vanishes_with_M(model, resampling):
    """Sec. IV D: without equilibration (theta = 0, condition (d)) and with
    constant population size (multinomial, condition (c)), configurational
    weighted averages converge to the exact ensemble average as M grows,
    while the plain average over runs keeps the finite-R bias.  Pool of
    runs partitioned into S groups of M (Sec. V A 2).  With nearest-integer
    resampling the population size fluctuates and the full weight of
    Eq. (appropriateWeight) carries the R_{k-1}/R factors that keep the
    same convergence."""
    L, R, K = 4, 4, 5
    beta_f = 0.3 if model == W.FM else 0.5
    d = W.run_desc(L, model, seed=3131, disorder_seed=12, R=R, R_cap=16 * R if resampling else R, theta=0, K=K,
                   beta_f=beta_f, resampling=resampling)
    pool = oracle.many_runs_obs(d, 60000)
    jR, jD = oracle.OracleRun(d).couplings()
    _, E, Mg = exact.enumerate_states(L, jR, jD)
    i = K - 1
    e_ex = exact.exact_from_enumeration(E, Mg, d["beta"][i], 16)["e"]
    lnZ_ex = exact.exact_from_enumeration(E, Mg, d["beta"][i], 16)["lnZ"]
    alive = pool[:, i]["status"] == oracle.OK
    e_runs = pool[alive, i]["sumE"] / (16.0 * pool[alive, i]["R_i"])
    plain_bias = e_runs.mean() - e_ex
    plain_err = e_runs.std() / math.sqrt(len(e_runs))
    assert abs(plain_bias) > 6 * plain_err         # finite R: PA alone is biased here

    def grouped(M):
        S = len(pool) // M
        We = np.empty(S)
        WF = np.empty(S)
        for s in range(S):
            o = oracle.weighted_average(pool[s * M:(s + 1) * M], d["beta"], 16, R, kind=0)
            We[s] = o["W_e"][i]
            WF[s] = o["minus_beta_WF"][i]
        return We.mean() - e_ex, We.std() / math.sqrt(S), WF.mean() - lnZ_ex

    b10, _, f10 = grouped(10)
    b100, _, f100 = grouped(100)
    b1000, err1000, f1000 = grouped(1000)
    assert abs(b1000) < abs(b100) < abs(b10) < abs(plain_bias)
    assert abs(b1000) < 0.25 * abs(plain_bias)
    assert abs(f1000) < abs(f10)              # -beta W[F] -> ln Z as M grows


def test_excluded_runs(small_pool):
    """Runs whose record carries a non-OK status are left out and counted."""
    d, obs = small_pool
    bad = obs.copy()
    bad["status"][3, 2:] = oracle.ERR_CAPACITY
    out = oracle.weighted_average(bad, d["beta"], 16, d["R"], kind=0)
    assert out["n_included"][0] == 64 and (out["n_included"][2:] == 63).all()
    ref = oracle.weighted_average(np.delete(obs, 3, axis=0), d["beta"], 16, d["R"], kind=0)
    assert np.allclose(out["W_e"][2:], ref["W_e"][2:], rtol=1e-13)


def test_weight_variance_prediction_small_spread():
    """var w ~ (exp(var beta F) - 1) / M^2 for log-normal weights, Eq. (varWpred);
    loose agreement for a large pool of small runs."""
    d = W.run_desc(4, W.FM, seed=606, R=64, theta=2, K=5, beta_f=0.5)
    obs = oracle.many_runs_obs(d, 400)
    out = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=1)
    for i in range(2, 5):
        assert out["var_w_pred"][i] > 0
        assert 0.5 < out["var_w"][i] / out["var_w_pred"][i] < 2.0
