"""Oracle pins for family statistics and the weighted overlap distribution,
CPU only.

* rho_t (Eq. (rho_t)) is computed in the oracle's measurement from its
  family histogram; here it is recomputed from the family labels of the
  returned population at every step, and checked against the integer record
  (sum c_k^2 / R_i).
* W[P(q)] (Eq. (W_conf_q)) is checked against identities that tie it to the
  separately coded overlap averages: it sums to one, and its first and second
  moments in |q| and q^2 are W[|q|] and W[q^2]; one run gives its own
  normalised histogram; identical runs give that of one run.
* The large-family exclusion (Sec. III D, Table I): a run with a family above
  R_i/2 carries no weight in the overlap averages (changing its overlap data
  changes nothing), runs without one are unaffected, and for two populations
  a large family in the other population also excludes the run.
"""
import numpy as np
import pytest

import oracle
import workloads as W

EXCL = oracle.EXCLUDE_LARGE_FAMILY


def ea_desc(m, L=4, R=40, K=9, theta=1, overlap=W.Q_INDEX_SHIFT, resampling=W.MULTINOMIAL):
    return W.run_desc(L, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x4400 + m, disorder_seed=W.DISORDER_SEED_BASE + 9,
                      R=R, theta=theta, K=K, beta_f=2.5, resampling=resampling, overlap=overlap, qhist=1)


@pytest.fixture(scope="module")
def pool():
    """12 runs on one 4x4 +-J sample, index-shift pairs, histograms kept."""
    runs = []
    for m in range(12):
        r = oracle.OracleRun(ea_desc(m))
        r.run_all()
        runs.append(r)
    obs = np.stack([r.obs()[0] for r in runs])        # [M, K]
    qh = np.stack([r.qhist()[0] for r in runs])        # [M, K, N+1]
    return runs, obs, qh


def q_values(N):
    return 1.0 - 2.0 * np.arange(N + 1) / N


def test_rho_t_from_family_labels():
    d = W.run_desc(8, W.EA_PMJ, seed=5, disorder_seed=6, R=300, theta=1, K=14, beta_f=3.0,
                   resampling=W.NEAREST_INT)
    run = oracle.OracleRun(d)
    for i in range(d["K"]):
        if i:
            run.step(i)
        _, _, fam, status = run.state(0)
        assert status == 0
        Ri = fam.shape[0]
        _, c = np.unique(fam, return_counts=True)
        n = c / Ri
        rho = Ri * np.sum(n * n)
        o = run.obs()[0, i]
        assert run.rho()[0, i] == pytest.approx(rho, rel=1e-12)
        assert o["famSumSq"] == int(np.sum(c.astype(np.int64) ** 2))
        assert run.rho()[0, i] == pytest.approx(o["famSumSq"] / o["R_i"], rel=1e-12)
        assert o["famMax"] == c.max() and o["nFam"] == len(c)


@pytest.mark.parametrize("kind", [0, 1, EXCL, 1 | EXCL])
def test_weighted_qhist_moments_are_the_overlap_averages(pool, kind):
    runs, obs, qh = pool
    N, R = 16, 40
    wp = oracle.weighted_qhist(obs, qh, N, R, kind=kind)
    wa = oracle.weighted_average(obs, ea_desc(0)["beta"], N, R, kind=kind)
    q = q_values(N)
    for i in range(obs.shape[1]):
        if np.isnan(wp[i]).any():
            assert np.isnan(wa["W_absq"][i])
            continue
        assert wp[i].sum() == pytest.approx(1.0, abs=1e-13)
        assert (wp[i] >= 0).all()
        assert np.dot(wp[i], np.abs(q)) == pytest.approx(wa["W_absq"][i], rel=1e-12, abs=1e-14)
        assert np.dot(wp[i], q * q) == pytest.approx(wa["W_q2"][i], rel=1e-12, abs=1e-14)


def test_weighted_qhist_single_and_identical_runs(pool):
    _, obs, qh = pool
    N, R = 16, 40
    one = oracle.weighted_qhist(obs[:1], qh[:1], N, R)
    np.testing.assert_allclose(one, qh[0] / obs[0]["nPairs"][:, None], rtol=1e-15, atol=0)
    rep = oracle.weighted_qhist(np.repeat(obs[:1], 4, 0), np.repeat(qh[:1], 4, 0), N, R)
    np.testing.assert_allclose(rep, one, rtol=1e-13, atol=1e-15)


def test_large_family_exclusion(pool):
    """Runs with a family above R_i/2 at temperature i carry no weight in the
    overlap averages there; the others are unaffected."""
    runs, obs, qh = pool
    N, R = 16, 40
    beta = ea_desc(0)["beta"]
    large = 2 * obs["famMax"] > obs["R_i"]
    assert large.any() and not large.all(), "the pool should have some large families and some not"
    base_p = oracle.weighted_qhist(obs, qh, N, R, kind=EXCL)
    base_a = oracle.weighted_average(obs, beta, N, R, kind=EXCL)
    # perturb the overlap data of every (run, i) with a large family
    obs2, qh2 = obs.copy(), qh.copy()
    obs2["sumAbsQ"][large] += 7
    obs2["sumQ2"][large] += 11
    qh2[large] = np.roll(qh2[large], 3, axis=-1)
    pert_p = oracle.weighted_qhist(obs2, qh2, N, R, kind=EXCL)
    pert_a = oracle.weighted_average(obs2, beta, N, R, kind=EXCL)
    np.testing.assert_array_equal(np.nan_to_num(pert_p, nan=-1), np.nan_to_num(base_p, nan=-1))
    np.testing.assert_array_equal(np.nan_to_num(pert_a["W_absq"], nan=-1), np.nan_to_num(base_a["W_absq"], nan=-1))
    # without the flag the same perturbation shows
    assert not np.allclose(oracle.weighted_qhist(obs2, qh2, N, R), oracle.weighted_qhist(obs, qh, N, R),
                           equal_nan=True)
    # temperatures with no large family: flag changes nothing
    plain = oracle.weighted_average(obs, beta, N, R, kind=0)
    for i in np.where(~large.any(axis=0))[0]:
        assert base_a["W_absq"][i] == plain["W_absq"][i]
    # the non-overlap averages never depend on the flag
    for f in ("W_e", "Wvar_c", "W_m", "minus_beta_WF", "n_included"):
        np.testing.assert_array_equal(base_a[f], plain[f])


def test_two_population_exclusion_uses_both_populations():
    d = ea_desc(0, L=4, R=24, K=10, overlap=W.Q_TWO_POP)
    runs = [oracle.OracleRun(W.with_(d, seed=d["seed"] + m)).run_all() for m in range(8)]
    o0 = np.stack([r.obs()[0] for r in runs])
    o1 = np.stack([r.obs()[1] for r in runs])
    fs = [oracle.family_stats(r.rho()[0], r.obs()[0], r.obs()[1]) for r in runs]
    for m, f in enumerate(fs):
        l0 = 2 * o0[m]["famMax"] > o0[m]["R_i"]
        l1 = 2 * o1[m]["famMax"] > o1[m]["R_i"]
        np.testing.assert_array_equal(f["large"], l0.astype(np.int32))
        np.testing.assert_array_equal(f["excluded"], (l0 | l1).astype(np.int32))
        np.testing.assert_allclose(f["rho_t"], o0[m]["famSumSq"] / o0[m]["R_i"], rtol=1e-12)
    only_other = np.array([[(f["excluded"][i] == 1 and f["large"][i] == 0) for i in range(d["K"])] for f in fs])
    assert only_other.any(), "some run should be excluded through its second population only"
    # the weighted |q| over pop 0 with obs_other drops exactly those runs: perturbing them changes nothing
    excl = np.array([f["excluded"] for f in fs]).astype(bool)
    o0b = o0.copy()
    o0b["sumAbsQ"][excl] += 5
    a = oracle.weighted_average(o0, d["beta"], 16, d["R"], kind=EXCL, obs_other=o1)
    b = oracle.weighted_average(o0b, d["beta"], 16, d["R"], kind=EXCL, obs_other=o1)
    np.testing.assert_array_equal(np.nan_to_num(a["W_absq"], nan=-1), np.nan_to_num(b["W_absq"], nan=-1))
