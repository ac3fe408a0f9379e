"""Oracle pins against exact statistical mechanics (CPU only).

Every check here compares the oracle with something it does not compute
itself: brute-force enumeration, the transfer matrix, Kaufman's finite-L
partition function, binomial/multinomial laws, or an identity of the paper.
All inputs are seeded, so each test is deterministic.
"""
import math

import numpy as np
import pytest

import exact
import oracle
import workloads as W


def _energy(s, L, jR, jD):
    """Energy of configurations s [R, N] by an independent vectorised loop."""
    s = s.astype(np.int64).reshape(-1, L, L)
    jR = jR.astype(np.int64).reshape(L, L)
    jD = jD.astype(np.int64).reshape(L, L)
    return -(jR * s * np.roll(s, -1, axis=2)).sum((1, 2)) - (jD * s * np.roll(s, -1, axis=1)).sum((1, 2))


# ------------------------------------------------------------------ step (i)

def test_initial_population_uniform_and_energies():
    """Step (i): spins i.i.d. uniform +-1 at beta_0 = 0; energies equal the
    Hamiltonian; family labels are 0..R-1; A_0 = ln Z(0) = N ln 2."""
    d = W.run_desc(8, W.EA_PMJ, seed=11, disorder_seed=5, R=700, theta=1, K=3, beta_f=0.1)
    r = oracle.OracleRun(d)
    s, E, f, st = r.state(0)
    jR, jD = r.couplings()
    assert st == 0 and s.shape == (700, 64)
    assert np.array_equal(E, _energy(s, 8, jR, jD))
    assert np.array_equal(f, np.arange(700))
    n = s.size
    z = (np.count_nonzero(s == 1) - n / 2) / math.sqrt(n / 4)
    assert abs(z) < 4.0
    # neighbouring sites and neighbouring replicas uncorrelated
    c1 = (s[:, :-1].astype(float) * s[:, 1:]).mean()
    c2 = (s[:-1].astype(float) * s[1:]).mean()
    assert abs(c1) < 4 / math.sqrt(s[:, 1:].size) and abs(c2) < 4 / math.sqrt(s[1:].size)
    o = r.obs()[0, 0]
    assert o["A"] == 64 * math.log(2.0)
    assert o["R_i"] == 700


def test_ea_couplings_half_negative():
    """+-J couplings drawn uniformly and independently (Sec. III A)."""
    d = W.run_desc(32, W.EA_PMJ, seed=1, disorder_seed=99, R=64, theta=0, K=2, beta_f=0.1)
    jR, jD = oracle.OracleRun(d).couplings()
    allj = np.concatenate([jR, jD])
    assert set(np.unique(allj)) == {-1, 1}
    z = (np.count_nonzero(allj == -1) - allj.size / 2) / math.sqrt(allj.size / 4)
    assert abs(z) < 4.0
    dFM = W.run_desc(8, W.FM, R=64, theta=0, K=2, beta_f=0.1)
    jR, jD = oracle.OracleRun(dFM).couplings()
    assert (jR == 1).all() and (jD == 1).all()


def test_energy_levels_spaced_by_four():
    """Any two configurations of one coupling set differ in energy by a
    multiple of 4, so k = (E - E_min)/4 is an integer in [0, N]."""
    _, E, _ = exact.enumerate_states(4, *oracle.OracleRun(
        W.run_desc(4, W.EA_PMJ, disorder_seed=3, R=8, theta=0, K=2, beta_f=0.1)).couplings())
    assert ((E - E.min()) % 4 == 0).all()
    assert (E.max() - E.min()) // 4 <= 16


# ----------------------------------------------------------------- step (iv)

def _fixed_beta_desc(L, model, beta, sweeps_steps, R, theta, seed=7, disorder_seed=1):
    """beta_0 = 0, then the same beta repeated: with nearest-integer
    resampling a step with dbeta = 0 has tau = 1 exactly (r_j = 1), so the
    later steps are pure checkerboard Metropolis sweeps at fixed beta."""
    return W.run_desc(L, model, seed=seed, disorder_seed=disorder_seed, R=R, R_cap=R + 64,
                      theta=theta, beta=[0.0] + [beta] * sweeps_steps,
                      resampling=W.NEAREST_INT)


@pytest.mark.parametrize("model,beta", [(W.FM, 0.3), (W.FM, 0.6), (W.EA_PMJ, 0.9)])
def test_sweeps_sample_boltzmann(model, beta):
    """Step (iv): checkerboard single-spin-flip Metropolis has the Boltzmann
    distribution as its stationary law (global balance, Sec. V A 1).  After
    many sweeps at fixed beta the population's energy histogram matches the
    exact one from enumeration (chi-square), and |M| matches for the FM."""
    L = 4
    d = _fixed_beta_desc(L, model, beta, sweeps_steps=12, R=4000, theta=4)
    r = oracle.OracleRun(d).run_all()
    assert r.energy_mismatches() == 0
    o = r.obs()[0]
    # dbeta = 0: tau_j = R / R_{i-1}; once R_{i-1} = R every replica is kept once
    first = int(np.argmax(o["R_i"][1:] == 4000)) + 1
    assert first < len(o) - 3 and (o["R_i"][first:] == 4000).all()
    assert (o["lnQ"][2:] == 0.0).all()         # Q = 1 exactly when dbeta = 0
    s, E, _, _ = r.state(0)
    jR, jD = r.couplings()
    _, Eall, Mall = exact.enumerate_states(L, jR, jD)
    p = exact.boltzmann(Eall, beta)
    levels = np.unique(Eall)
    pe = np.array([p[Eall == e].sum() for e in levels])
    cnt = np.array([(E == e).sum() for e in levels])
    keep = pe * len(E) > 5
    exp_ = pe[keep] * len(E)
    obs_ = cnt[keep]
    chi2 = ((obs_ - exp_) ** 2 / exp_).sum() + 0.0
    dof = keep.sum() - 1
    # replicas decorrelate over 48 sweeps at these temperatures: loose bound
    assert chi2 < dof + 8 * math.sqrt(2 * dof) + 10, (chi2, dof)
    if model == W.FM:
        m_ex = (p * np.abs(Mall)).sum() / 16
        m = np.abs(s.sum(1)).mean() / 16
        assert abs(m - m_ex) < 5 * np.abs(s.sum(1) / 16).std() / math.sqrt(len(E))


def test_acceptance_rate_matches_threshold():
    """A single colour update from a fully aligned FM state: every attempted
    flip has dE = 8 and is accepted with probability T(beta, 8)/2^32."""
    beta = 0.2
    d = W.run_desc(4, W.FM, seed=21, R=4096, R_cap=4160, theta=1, beta=[0.0, 50.0, 50.0, beta],
                   resampling=W.NEAREST_INT)
    r = oracle.OracleRun(d)
    # anneal to a huge beta: the population collapses onto the two ground states
    for i in (1, 2):
        r.step(i)
    s, _, _, _ = r.state(0)
    assert (np.abs(s.sum(1)) == 16).all()
    r.anneal_step(3)
    r.resample(3)
    s0, _, _, _ = r.state(0)
    r.sweep(3)
    s1, _, _, _ = r.state(0)
    # colour-0 sites see an aligned neighbourhood (dE = 8); count their flips
    L = 4
    col0 = [n for n in range(16) if ((n % L + n // L) & 1) == 0]
    flips = (s0[:, col0] != s1[:, col0]).sum()
    trials = s0.shape[0] * len(col0)
    p = oracle.sweep_threshold(beta, 8) / 2 ** 32
    z = (flips - trials * p) / math.sqrt(trials * p * (1 - p))
    assert abs(z) < 4.0


# ------------------------------------------------------------ steps (ii)-(iii)

def test_nearest_integer_counts():
    """Nearest-integer resampling (Sec. II B): r_j in {floor tau, ceil tau}
    with tau_j = R X_j / S_X, sum r = R_i, and E[r_j] = tau_j (z-score of
    sum (r - tau) over many replicas and steps)."""
    d = W.run_desc(8, W.FM, seed=5, R=600, R_cap=900, theta=2, K=30, beta_f=1.2,
                   resampling=W.NEAREST_INT)
    r = oracle.OracleRun(d)
    dev = 0.0
    var = 0.0
    for i in range(1, 30):
        r.anneal_step(i)
        r.resample(i)
        cnt, X, SX = r.counts(0)
        RX = [600 * int(x) for x in X]
        lo = np.array([v // SX for v in RX])
        frac = np.array([(v % SX) / SX for v in RX])
        assert ((cnt == lo) | (cnt == lo + 1)).all()
        assert cnt.sum() == r.state(0)[1].shape[0]
        assert sum(int(x) for x in X) == SX
        dev += (cnt - lo - frac).sum()
        var += (frac * (1 - frac)).sum()
        r.sweep(i)
        r.measure(i)
    assert abs(dev) < 4.5 * math.sqrt(var)


def test_multinomial_counts_chi_square():
    """Multinomial resampling: sum r = R and r ~ Multinomial(R, X/S_X): the
    Pearson statistic over parents of the pooled counts stays below its
    dof + 5 sigma."""
    d = W.run_desc(6, W.FM, seed=17, R=400, theta=1, K=12, beta_f=1.5)
    r = oracle.OracleRun(d)
    chi2 = 0.0
    dof = 0
    for i in range(1, 12):
        r.anneal_step(i)
        r.resample(i)
        cnt, X, SX = r.counts(0)
        assert cnt.sum() == 400
        p = X.astype(np.float64) / SX
        e = 400 * p
        keep = e > 2
        chi2 += ((cnt[keep] - e[keep]) ** 2 / e[keep]).sum()
        dof += keep.sum()
        assert cnt[X == 0].sum() == 0
        r.sweep(i)
        r.measure(i)
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_copies_contiguous_and_faithful():
    """Copies of one parent are placed next to each other: family labels
    non-decreasing, each child equals its parent (spins and energy)."""
    d = W.run_desc(8, W.EA_PMJ, seed=3, R=300, R_cap=500, theta=1, K=8, beta_f=2.0,
                   resampling=W.NEAREST_INT)
    r = oracle.OracleRun(d)
    for i in range(1, 8):
        r.anneal_step(i)
        s_par, E_par, f_par, _ = r.state(0)
        r.resample(i)
        cnt, _, _ = r.counts(0)
        s_ch, E_ch, f_ch, _ = r.state(0)
        parent = np.repeat(np.arange(len(cnt)), cnt)
        assert np.array_equal(s_ch, s_par[parent])
        assert np.array_equal(E_ch, E_par[parent])
        assert np.array_equal(f_ch, f_par[parent])
        assert (np.diff(f_ch) >= 0).all()
        r.sweep(i)
        r.measure(i)


# -------------------------------------------- free energy: unbiasedness (T4)

@pytest.mark.parametrize("model,theta", [(W.FM, 0), (W.FM, 1), (W.EA_PMJ, 0), (W.EA_PMJ, 2)])
def test_partition_function_estimate_unbiased(model, theta):
    """With constant population size (multinomial) the product of the Q_k is
    an unbiased estimate of Z(beta_i)/Z(beta_0) for any R (Sec. IV D: the
    proof's numerator equals C_i/C_0; it also holds with equilibration
    moves that leave the target invariant).  Mean over many runs of
    exp(A_i - N ln 2) versus exact Z(beta_i)/2^N from enumeration."""
    L, R, K = 4, 8, 6
    d = W.run_desc(L, model, seed=1000 + theta, disorder_seed=4, R=R, theta=theta, K=K,
                   beta_f=0.75 if model == W.FM else 1.2)
    M = 40000
    A, _, Rr = oracle.many_runs(d, M)
    assert (Rr == R).all()
    jR, jD = oracle.OracleRun(d).couplings()
    _, E, Mg = exact.enumerate_states(L, jR, jD)
    for i in range(1, K):
        lnZ = exact.exact_from_enumeration(E, Mg, d["beta"][i], 16)["lnZ"]
        ratio = np.exp(A[:, i] - lnZ)          # unbiased estimate of 1
        z = (ratio.mean() - 1.0) / (ratio.std() / math.sqrt(M))
        assert abs(z) < 4.5, (i, ratio.mean(), z)


# ------------------------------------------------ whole runs versus exact (T3)

@pytest.fixture(scope="module")
def fm_L8_runs():
    """16 independent PA runs of the L=8 ferromagnet (R=500, theta=10,
    beta 0 -> 1 in 51 points, multinomial)."""
    d = W.run_desc(8, W.FM, seed=0x5EED0000, R=500, theta=10, K=51, beta_f=1.0)
    return d, oracle.many_runs_obs(d, 16)


def test_pa_energy_heat_capacity_free_energy_vs_kaufman(fm_L8_runs):
    """Population averages e, c and the free-energy estimator -beta F = A
    (Eqs. (e), (c), (F)) agree with Kaufman's exact finite-L results within
    statistical errors over 16 runs (plus a small allowance for PA's
    systematic error at R = 500)."""
    d, obs = fm_L8_runs
    N = 64
    for i in (5, 15, 22, 30, 40, 50):
        beta = d["beta"][i]
        lnZ, e_ex, c_ex = exact.kaufman_thermo(8, beta)
        o = obs[:, i]
        R = o["R_i"].astype(np.float64)
        e = o["sumE"] / (N * R)
        var = (R * o["sumE2"].astype(np.float64) - o["sumE"].astype(np.float64) ** 2)
        c = beta ** 2 * var / (N * R * R)
        A = o["A"]
        for est, ex, tol in ((e, e_ex, 0.004), (c, c_ex, 0.06), (A / N, lnZ / N, 0.002)):
            err = est.std(ddof=1) / math.sqrt(len(est))
            assert abs(est.mean() - ex) < 4.5 * err + tol, (i, est.mean(), ex, err)


def test_pa_magnetisation_vs_transfer_matrix(fm_L8_runs):
    """|m| and m^2 (Eq. (m)) agree with the exact magnetisation distribution
    of the L = 8 torus from the transfer matrix."""
    d, obs = fm_L8_runs
    N = 64
    for i in (10, 22, 35, 50):
        beta = d["beta"][i]
        Mv, p = exact.fm_transfer_M_distribution(8, beta)
        m_ex = (p * np.abs(Mv)).sum() / N
        m2_ex = (p * Mv.astype(float) ** 2).sum() / N ** 2
        o = obs[:, i]
        R = o["R_i"].astype(np.float64)
        m = o["sumAbsM"] / (N * R)
        m2 = o["sumM2"] / (N * N * R)
        for est, ex in ((m, m_ex), (m2, m2_ex)):
            err = est.std(ddof=1) / math.sqrt(len(est))
            assert abs(est.mean() - ex) < 4.5 * err + 0.01, (i, est.mean(), ex, err)


def test_free_energy_limit_ground_state():
    """For the 2D FM, f -> -z/2 = -2 as beta -> infinity (Sec. III C, App. A)."""
    d = W.run_desc(8, W.FM, seed=9, R=300, theta=5, beta=list(np.linspace(0, 1, 41)) +
                   [1.5, 2.5, 4.0, 6.0, 9.0, 14.0, 20.0])
    o = oracle.OracleRun(d).run_all().obs()[0]
    f = -o["A"][-1] / (20.0 * 64)
    assert abs(f + 2.0) < 2e-3


# ------------------------------------------------------------------ overlaps

def test_overlaps_index_shift_and_two_populations():
    """Overlap sums (Sec. III D) recomputed from the returned configurations:
    index-shift pairs (j, j + floor(R_i/2)) and two-population pairs."""
    d = W.run_desc(6, W.EA_PMJ, seed=2, disorder_seed=8, R=301, R_cap=420, theta=2, K=6,
                   beta_f=1.5, resampling=W.NEAREST_INT, overlap=W.Q_INDEX_SHIFT, qhist=1)
    r = oracle.OracleRun(d).run_all()
    s, _, f, _ = r.state(0)
    o = r.obs()[0, -1]
    L, N = 6, 36
    h = len(s) // 2
    a, b = s[:h].astype(np.int64), s[h:2 * h].astype(np.int64)
    Q = (a * b).sum(1)

    def links(x):
        x = x.reshape(-1, L, L)
        return np.concatenate([(x * np.roll(x, -1, 2)).reshape(len(x), -1),
                               (x * np.roll(x, -1, 1)).reshape(len(x), -1)], 1)
    Ql = (links(a) * links(b)).sum(1)
    assert o["nPairs"] == h
    assert o["sumQ"] == Q.sum() and o["sumAbsQ"] == np.abs(Q).sum() and o["sumQ2"] == (Q * Q).sum()
    assert o["sumQl"] == Ql.sum() and o["sumQl2"] == (Ql * Ql).sum()
    hist = r.qhist()[0, -1]
    assert np.array_equal(hist, np.bincount((N - Q) // 2, minlength=N + 1))
    c = np.bincount(f)
    assert o["famSumSq"] == (c.astype(np.int64) ** 2).sum() and o["famMax"] == c.max()
    assert o["nFam"] == np.count_nonzero(c)

    d2 = W.with_(d, overlap=W.Q_TWO_POP)
    r2 = oracle.OracleRun(d2).run_all()
    sA, _, _, _ = r2.state(0)
    sB, _, _, _ = r2.state(1)
    m = min(len(sA), len(sB))
    Q = (sA[:m].astype(np.int64) * sB[:m]).sum(1)
    for pop in (0, 1):
        o = r2.obs()[pop, -1]
        assert o["nPairs"] == m and o["sumQ"] == Q.sum() and o["sumQ2"] == (Q * Q).sum()
    assert not np.array_equal(sA[:m], sB[:m])       # populations are independent


def test_two_population_overlap_distribution_vs_exact():
    """Two independent populations on one 4x4 +-J sample: the pooled overlap
    histogram at the final beta matches the exact P(q) from the
    Walsh-Hadamard autocorrelation of the Boltzmann law."""
    beta = 0.8
    d = W.run_desc(4, W.EA_PMJ, seed=44, disorder_seed=6, R=3000, R_cap=3100, theta=5,
                   beta=[0.0, 0.2, 0.4, 0.6, beta, beta, beta, beta], resampling=W.NEAREST_INT,
                   overlap=W.Q_TWO_POP, qhist=1)
    r = oracle.OracleRun(d).run_all()
    hist = r.qhist()[0, -1].astype(np.float64)
    jR, jD = r.couplings()
    S, E, _ = exact.enumerate_states(4, jR, jD)
    Pq, _ = exact.overlap_distributions(S, E, 4, beta)
    n = hist.sum()
    keep = Pq * n > 5
    chi2 = ((hist[keep] - n * Pq[keep]) ** 2 / (n * Pq[keep])).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 8 * math.sqrt(2 * dof) + 10, (chi2, dof)


# -------------------------------------------------------- failure handling

def test_capacity_overflow_freezes_run():
    """Nearest-integer with R_cap = R: a step whose population would exceed
    the capacity marks the run CAPACITY and freezes it; later records carry
    the status and zero sums."""
    d = W.run_desc(4, W.FM, seed=1, R=64, R_cap=64, theta=0, K=20, beta_f=8.0,
                   resampling=W.NEAREST_INT)
    o = oracle.OracleRun(d).run_all().obs()[0]
    bad = np.nonzero(o["status"] != 0)[0]
    assert len(bad) > 0
    first = bad[0]
    assert (o["status"][first:] == oracle.ERR_CAPACITY).all()
    assert (o["R_i"][first:] == 0).all() and (o["status"][:first] == 0).all()


def test_out_of_order_calls_rejected():
    d = W.run_desc(4, W.FM, R=64, theta=1, K=4, beta_f=0.5)
    r = oracle.OracleRun(d)
    assert r.resample(1) == oracle.ERR_STATE
    assert r.anneal_step(2) == oracle.ERR_STATE
    assert r.anneal_step(1) == 0
    assert r.sweep(1) == oracle.ERR_STATE
    assert r.resample(1) == 0 and r.sweep(1) == 0 and r.measure(1) == 0
