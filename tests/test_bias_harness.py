"""Pins for the bias-versus-M harness (paper_2207_05535_amd/bias.py), CPU only.

* Exact references: e, c, f from the density of states equal Kaufman's
  closed form (tests/exact.py) at L = 8 (density of states from the oracle).
* The jackknife error of a mean equals the textbook s / sqrt(n) exactly; the
  bootstrap error of a mean approaches s sqrt((n-1)/n) / sqrt(n).
* The power-law fit recovers a and b from exact data, and its error equals
  the closed-form standard error of a weighted straight-line fit; the
  a + b / beta fit recovers a and b from exact data.
* RMSD and Wang's estimate follow their definitions on hand-made numbers.
"""
import math

import numpy as np
import pytest

import exact
import oracle
from paper_2207_05535_amd import bias


@pytest.mark.parametrize("beta", [0.2, 0.4407, 0.7])
def test_exact_fm_matches_kaufman(beta):
    L = 8
    got = bias.exact_fm(oracle.exact_dos(L), L, beta)
    lnZ, e, c = exact.kaufman_thermo(L, beta)
    assert got["lnZ"] == pytest.approx(float(lnZ), rel=1e-13)
    assert got["e"] == pytest.approx(float(e), rel=1e-9)
    assert got["c"] == pytest.approx(float(c), rel=1e-7)
    assert got["f"] == pytest.approx(-float(lnZ) / (beta * L * L), rel=1e-13)


def test_jackknife_of_the_mean_is_the_standard_error():
    x = np.random.default_rng(1).normal(size=(37, 3))
    est, err = bias.jackknife(x)
    np.testing.assert_allclose(est, x.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(err, x.std(axis=0, ddof=1) / math.sqrt(37), rtol=1e-12)


def test_bootstrap_of_the_mean():
    x = np.random.default_rng(2).exponential(size=400)
    est, err = bias.bootstrap(x, n_boot=4000, seed=3)
    assert est == pytest.approx(x.mean())
    want = x.std(ddof=0) / math.sqrt(len(x))
    assert err == pytest.approx(want, rel=0.05)


def test_power_law_fit():
    M = np.array([1, 2, 4, 8, 16, 32.0])
    y = 0.3 * M ** -0.8
    sig = 0.05 * y * np.array([1, 2, 1, 3, 1, 2.0])
    a, b, sb = bias.fit_power_law(M, y, sig)
    assert a == pytest.approx(0.3, rel=1e-12) and b == pytest.approx(0.8, rel=1e-12)
    # closed-form slope error of a weighted straight line: 1 / sqrt(sum w (x - xbar_w)^2)
    w = 1.0 / (sig / y) ** 2
    x = np.log(M)
    xbar = (w * x).sum() / w.sum()
    assert sb == pytest.approx(1.0 / math.sqrt((w * (x - xbar) ** 2).sum()), rel=1e-12)


def test_inverse_beta_fit():
    beta = np.linspace(0.6, 1.0, 9)
    a, b = bias.fit_a_plus_b_over_beta(beta, 0.01 - 0.002 / beta)
    assert a == pytest.approx(0.01, rel=1e-12) and b == pytest.approx(-0.002, rel=1e-10)


def test_rmsd_and_wang_estimate():
    assert bias.rmsd(3.0, 16.0) == pytest.approx(5.0)
    # F = N f: (beta/2) var F / N with var F = N^2 var f
    assert bias.wang_f_bias(0.5, 2.0e-6, 100) == pytest.approx(0.5 / 2 * (100 ** 2 * 2.0e-6) / 100)
