"""Oracle pins for the theta = infinity limit (Sec. V C), CPU only.

* The exact density of states of the periodic ferromagnet equals brute-force
  enumeration at L = 4, and at L = 6 and 8 reproduces Kaufman's closed-form
  partition function (written independently in tests/exact.py) to 25 digits
  at several temperatures; it sums to 2^N.
* The density of states of the product formula (oracle/dos.py), which the
  theta = infinity limit uses beyond L = 8, equals the transfer matrix's at
  L = 4, 6, 8, and at L = 10, 12, 16 sums to 2^N, is symmetric and
  reproduces Kaufman's partition function to 25 digits.
* A theta = infinity run draws every replica's energy from the exact
  distribution at beta_i: the population's energy histogram after the draw
  passes a chi-square test against g(E) exp(-beta E) / Z.
* The free-energy estimate stays unbiased in this limit: the mean over many
  runs of exp(A_i - N ln 2) equals Z(beta_i) / 2^N (Sec. IV D).
* With theta = infinity the recorded magnetisation sums are zero (energies
  only) and the recorded energy sums are those of the drawn energies.
"""
import math

import numpy as np
import pytest

import exact
import oracle
import workloads as W

THETA_INF = -1


def energies(L):
    N = L * L
    return np.array([-2 * N + 4 * m for m in range(N + 1)])


def test_dos_equals_enumeration_at_L4():
    _, E, _ = exact.enumerate_states(4)
    counts = np.bincount((E + 32) // 4, minlength=17)
    assert oracle.exact_dos(4) == [int(c) for c in counts]


@pytest.mark.parametrize("L", [6, 8])
def test_dos_reproduces_kaufman(L):
    import mpmath as mp
    g = oracle.exact_dos(L)
    N = L * L
    assert sum(g) == 2 ** N
    assert g == g[::-1]                          # E <-> -E on the bipartite lattice
    with mp.workdps(50):
        for beta in (0.1, 0.3, 0.4407, 0.6, 1.0):
            Z = mp.fsum(mp.mpf(gm) * mp.exp(-mp.mpf(beta) * (-2 * N + 4 * m)) for m, gm in enumerate(g))
            ref = exact.kaufman_lnZ(L, beta, dps=50)
            assert abs(mp.log(Z) - ref) < mp.mpf(10) ** -25 * abs(ref), (L, beta)


def test_product_formula_dos_equals_transfer_matrix():
    from oracle import dos
    for L in (4, 6, 8):
        assert list(dos.fm_dos(L)) == oracle.exact_dos(L), L


@pytest.mark.parametrize("L", [10, 12, 16])
def test_product_formula_dos_reproduces_kaufman(L):
    import mpmath as mp
    from oracle import dos
    g = list(dos.fm_dos(L))
    N = L * L
    assert sum(g) == 2 ** N and min(g) >= 0
    assert g == g[::-1]
    assert g[0] == 2 and g[1] == 0 and g[2] == 2 * N     # ground states; one flipped spin costs 4 bonds
    with mp.workdps(60):
        for beta in (0.05, 0.3, 0.4407, 0.6, 1.2):
            Z = mp.fsum(mp.mpf(gm) * mp.exp(-mp.mpf(beta) * (-2 * N + 4 * m)) for m, gm in enumerate(g))
            ref = exact.kaufman_lnZ(L, beta, dps=60)
            assert abs(mp.log(Z) - ref) < mp.mpf(10) ** -25 * abs(ref), (L, beta)


@pytest.mark.parametrize("L,R", [(4, 20000), (16, 20000)])
def test_theta_infinity_draws_the_exact_energy_law(L, R):
    from scipy import stats
    from oracle import dos
    d = W.run_desc(L, W.FM, seed=0x1F0 + L, R=R, theta=THETA_INF, K=5, beta_f=0.8 if L == 4 else 0.44)
    run = oracle.OracleRun(d)
    g = np.array(dos.fm_dos_doubles(L), np.float64)
    Es = energies(L)
    for i in range(1, d["K"]):
        run.step(i)
        _, E, _, st = run.state(0)
        assert st == 0
        p = g * np.exp(-d["beta"][i] * (Es - Es[0]))
        p /= p.sum()
        obs = np.bincount((E - Es[0]) // 4, minlength=L * L + 1)
        keep = p * len(E) >= 5
        exp_ = p[keep] * len(E)
        o = obs[keep].astype(np.float64)
        o_rest, e_rest = len(E) - o.sum(), len(E) - exp_.sum()
        chi2 = ((o - exp_) ** 2 / exp_).sum() + ((o_rest - e_rest) ** 2 / e_rest if e_rest > 1e-9 else 0.0)
        assert stats.chi2.sf(chi2, keep.sum()) > 1e-4, (i, chi2)
        rec = run.obs()[0, i]
        assert rec["sumE"] == E.sum() and rec["sumE2"] == (E.astype(np.int64) ** 2).sum()
        assert rec["sumAbsM"] == 0 and rec["sumM2"] == 0 and rec["nPairs"] == 0


def test_theta_infinity_free_energy_unbiased():
    L, R, K, M = 4, 8, 6, 30000
    d = W.run_desc(L, W.FM, seed=0x2F0, R=R, theta=THETA_INF, K=K, beta_f=0.75)
    A, _, Rr = oracle.many_runs(d, M)
    assert (Rr == R).all()
    _, E, Mg = exact.enumerate_states(L)
    for i in range(1, K):
        lnZ = exact.exact_from_enumeration(E, Mg, d["beta"][i], 16)["lnZ"]
        ratio = np.exp(A[:, i] - lnZ)
        z = (ratio.mean() - 1.0) / (ratio.std() / math.sqrt(M))
        assert abs(z) < 4.5, (i, ratio.mean(), z)


def test_theta_infinity_rejected_outside_its_domain():
    for bad in (dict(model=W.EA_PMJ), dict(L=32), dict(overlap=W.Q_INDEX_SHIFT)):
        kw = dict(L=4, model=W.FM, overlap=W.Q_NONE)
        kw.update(bad)
        d = W.run_desc(kw["L"], kw["model"], R=10, theta=THETA_INF, K=3, beta_f=0.5, overlap=kw["overlap"])
        with pytest.raises(ValueError):
            oracle.OracleRun(d)
