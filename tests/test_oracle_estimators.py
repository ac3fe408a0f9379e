"""Oracle pins for the weighted-average estimators against exact values
(CPU only).

* The full free-energy weight, Eq. (appropriateWeight): with nearest-integer
  resampling the population size fluctuates, and the weight's product of
  R_{k-1}/R factors is what keeps it an unbiased estimate of the partition
  function.  Thinking of normalised PA as unnormalised PA rescaled by
  R / (R_{k-1} Q_k) at every step (Sec. IV A), the estimated size of the
  unnormalised population, R_i prod_{k<=i} (R_{k-1} Q_k / R), has expectation
  R Z(beta_i) / Z(beta_0) for Metropolis moves that keep the Boltzmann law
  invariant; with A_i = sum_k ln Q_k + N ln 2 that is
  E[exp(a_i - ln R - N ln 2)] = Z(beta_i) / 2^N for a_i the full log-weight.
  Runs whose population died out contribute zero.
* The susceptibility, Eq. (chi), and its weighted variance estimator,
  Eq. (Wvar_Chi): W_var[chi] = beta N (W[m^2] - W[|m|]^2) exactly, and both
  the single-run estimator and W_var[chi] agree with the exact chi of the
  4 x 4 torus (enumeration) and of the 8 x 8 torus (transfer matrix).
* The link overlap, with q_l = (1/2N) sum over the 2N bonds: two
  independent populations on a 4 x 4 +-J sample give W[q_l] equal to the
  exact <q_l> of two independent Boltzmann replicas (Walsh-Hadamard
  autocorrelation of the Boltzmann law); likewise W[|q|] and W[q^2].
"""
import math

import numpy as np
import pytest

import exact
import oracle
import workloads as W


def _z_scores(samples, target):
    n = len(samples)
    return (samples.mean() - target) / (samples.std(ddof=1) / math.sqrt(n))


@pytest.mark.parametrize("model,theta,M,K,beta_f", [
    (W.FM, 1, 200_000, 9, 0.8),
    (W.EA_PMJ, 1, 200_000, 9, 0.8),
    (W.FM, 0, 100_000, 5, 0.4),
    (W.EA_PMJ, 0, 100_000, 5, 0.4),
])
def test_full_weight_estimates_partition_function(model, theta, M, K, beta_f):
    """Mean over M nearest-integer runs (R = 4) of exp(a_i - ln R - N ln 2),
    a_i the oracle's full log-weight, equals Z(beta_i)/2^N from enumeration
    at every temperature.  Dropping the R_{k-1}/R product, or taking R_k in
    its place, moves the mean by many standard errors at these sizes."""
    L, N, R = 4, 16, 4
    d = W.run_desc(L, model, seed=0xF011 + 17 * model + theta, disorder_seed=7, R=R, R_cap=16 * R,
                   theta=theta, K=K, beta_f=beta_f, resampling=W.NEAREST_INT)
    jR, jD = oracle.OracleRun(d).couplings()
    _, E, Mg = exact.enumerate_states(L, jR, jD)
    acc = np.zeros((0, K))
    chunk = 50_000
    for c0 in range(0, M, chunk):
        obs = oracle.many_runs_obs(W.with_(d, seed=d["seed"] + c0 * 1000003), chunk)
        st = obs["status"]
        # a run can only stop by dying out here (R_cap is never reached)
        assert np.all((st == oracle.OK) | (st == oracle.ERR_NUMERIC))
        assert obs["R_i"].max() < d["R_cap"]
        a = oracle.log_weights(obs, R, kind=0)
        est = np.where(np.isfinite(a), np.exp(np.where(np.isfinite(a), a, 0.0) - math.log(R) - N * math.log(2)), 0.0)
        acc = np.concatenate([acc, est])
    for i in range(K):
        lnZ = exact.exact_from_enumeration(E, Mg, d["beta"][i], N)["lnZ"]
        target = math.exp(lnZ - N * math.log(2))
        if i == 0:
            assert np.allclose(acc[:, 0], 1.0, rtol=1e-14)
            continue
        z = _z_scores(acc[:, i], target)
        assert abs(z) < 4.5, (i, acc[:, i].mean(), target, z)


def test_full_weight_is_what_the_weighted_average_uses():
    """W[e] from the oracle's weighted average equals sum_m w_m e_m with
    w = softmax of the exported log-weights (full and simplified), and the
    two kinds differ once R_i fluctuates."""
    d = W.run_desc(4, W.FM, seed=41, R=6, R_cap=60, theta=1, K=8, beta_f=0.9, resampling=W.NEAREST_INT)
    obs = oracle.many_runs_obs(d, 50)
    assert (obs["status"] == oracle.OK).all()
    e = obs["sumE"] / (16.0 * obs["R_i"])
    res = {}
    for kind in (0, 1):
        a = oracle.log_weights(obs, d["R"], kind=kind)
        w = np.exp(a - a.max(axis=0))
        w /= w.sum(axis=0)
        out = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=kind)
        assert np.allclose(out["W_e"], (w * e).sum(axis=0), rtol=1e-12, atol=1e-14)
        res[kind] = a
    # simplified: ln R_i + A_i; full adds sum_{k=1..i} ln(R_{k-1}/R)
    Ri = obs["R_i"].astype(np.float64)
    assert np.allclose(res[1], np.log(Ri) + obs["A"], rtol=1e-14)
    corr = np.concatenate([np.zeros((50, 1)), np.cumsum(np.log(Ri[:, :-1] / d["R"]), axis=1)], axis=1)
    assert np.allclose(res[0], res[1] + corr, rtol=1e-13, atol=1e-13)
    assert np.abs(corr[:, -1]).max() > 0.1


@pytest.mark.parametrize("resampling", [W.MULTINOMIAL, W.NEAREST_INT])
def test_weighted_variance_of_chi_identity(resampling):
    """W_var[chi] = beta N (W[m^2] - W[|m|]^2), Eq. (Wvar_Chi), for both weight
    kinds, and the per-run chi (M = 1) equals beta N (m2 - m^2) of that run."""
    R = 10
    d = W.run_desc(4, W.FM, seed=8, R=R, R_cap=R if resampling == W.MULTINOMIAL else 40, theta=1, K=8,
                   beta_f=1.2, resampling=resampling)
    obs = oracle.many_runs_obs(d, 30)
    b = np.asarray(d["beta"])
    for kind in (0, 1):
        out = oracle.weighted_average(obs, d["beta"], 16, d["R"], kind=kind)
        direct = b * 16 * (out["W_m2"] - out["W_m"] ** 2)
        assert np.allclose(out["Wvar_chi"], direct, rtol=1e-9, atol=1e-12)
    one = oracle.weighted_average(obs[:1], d["beta"], 16, d["R"], kind=0)
    o = obs[0]
    m = o["sumAbsM"] / (16.0 * o["R_i"])
    m2 = o["sumM2"] / (256.0 * o["R_i"])
    assert np.allclose(one["Wconf_chi"], b * 16 * (m2 - m * m), rtol=1e-9, atol=1e-12)


def _chi_vs_exact(d, n_runs, exact_chi, idx, tol):
    obs = oracle.many_runs_obs(d, n_runs)
    N = d["L"] ** 2
    per_run = np.stack([oracle.weighted_average(obs[m:m + 1], d["beta"], N, d["R"], kind=0)["Wconf_chi"]
                        for m in range(n_runs)])
    pooled = oracle.weighted_average(obs, d["beta"], N, d["R"], kind=0)
    for i in idx:
        ex = exact_chi(d["beta"][i])
        est = per_run[:, i]
        err = est.std(ddof=1) / math.sqrt(n_runs)
        assert abs(est.mean() - ex) < 4.5 * err + tol * ex, ("chi", i, est.mean(), ex, err)
        assert abs(pooled["Wvar_chi"][i] - ex) < 4.5 * err + tol * ex, ("Wvar_chi", i, pooled["Wvar_chi"][i], ex)
        # a slip by a factor of beta or N would move these by far more
        assert 4.5 * err + tol * ex < 0.3 * ex


def test_chi_vs_enumeration_L4():
    """Eq. (chi) per run and W_var[chi] versus the exact chi of the 4 x 4 torus."""
    d = W.run_desc(4, W.FM, seed=0xC41, R=4000, theta=10, K=13, beta_f=0.9)
    _, E, Mg = exact.enumerate_states(4)
    _chi_vs_exact(d, 8, lambda b: exact.exact_from_enumeration(E, Mg, b, 16)["chi"], (3, 6, 9), 0.01)


def test_chi_vs_transfer_matrix_L8():
    """Eq. (chi) per run and W_var[chi] versus the exact chi of the 8 x 8 torus
    from the magnetisation-resolved transfer matrix."""
    d = W.run_desc(8, W.FM, seed=0xC48, R=3000, theta=10, K=16, beta_f=0.6)

    def chi_tm(b):
        Mv, p = exact.fm_transfer_M_distribution(8, b)
        m = (p * np.abs(Mv)).sum() / 64
        m2 = (p * Mv.astype(float) ** 2).sum() / 64 ** 2
        return b * 64 * (m2 - m * m)
    _chi_vs_exact(d, 8, chi_tm, (5, 11, 15), 0.02)


def test_link_and_spin_overlaps_vs_exact():
    """Two independent populations on a 4 x 4 +-J sample: W[q_l], W[|q|] and
    W[q^2] (per run, M = 1, and pooled) agree with the exact values for two
    independent Boltzmann replicas."""
    beta_f, K = 1.2, 13
    d = W.run_desc(4, W.EA_PMJ, seed=0x91, disorder_seed=6, R=3000, R_cap=3200, theta=10, K=K,
                   beta_f=beta_f, resampling=W.NEAREST_INT, overlap=W.Q_TWO_POP)
    runs = [oracle.OracleRun(W.with_(d, seed=d["seed"] + m)).run_all() for m in range(6)]
    jR, jD = runs[0].couplings()
    S, E, _ = exact.enumerate_states(4, jR, jD)
    obs0 = np.stack([r.obs()[0] for r in runs])
    obs1 = np.stack([r.obs()[1] for r in runs])
    N = 16
    for i in (4, 8, 12):
        b = d["beta"][i]
        Pq, Pql = exact.overlap_distributions(S, E, 4, b)
        q = (N - 2 * np.arange(N + 1)) / N
        ex = {"W_absq": (Pq * np.abs(q)).sum(), "W_q2": (Pq * q * q).sum(),
              "W_ql": sum(v * p for v, p in Pql.items()) / (2 * N)}
        per = {f: [] for f in ex}
        for m in range(len(runs)):
            o = oracle.weighted_average(obs0[m:m + 1], d["beta"], N, d["R"], kind=0, obs_other=obs1[m:m + 1])
            for f in ex:
                per[f].append(o[f][i])
        pooled = oracle.weighted_average(obs0, d["beta"], N, d["R"], kind=0, obs_other=obs1)
        for f, v in ex.items():
            est = np.asarray(per[f])
            err = est.std(ddof=1) / math.sqrt(len(est))
            assert abs(est.mean() - v) < 4.5 * err + 0.005, (f, i, est.mean(), v, err)
            assert abs(pooled[f][i] - v) < 4.5 * err + 0.005, (f, i, pooled[f][i], v)
            # a normalisation by N instead of 2N (or N^2 for N) would be far outside
            assert 4.5 * err + 0.005 < 0.3 * v
