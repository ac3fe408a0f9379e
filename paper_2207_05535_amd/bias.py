"""Bias-versus-M analysis of weighted averages (Sec. V B; Table III,
Figs. 2 and 11), on top of the device's grouped weighted averages.

A pool of independent runs of one model is split into S = floor(pool / M)
groups of M runs (``Context.weighted_average(M)`` groups consecutive runs;
runs with different seeds are exchangeable, so this is a random partition
in distribution).  For each M the S weighted estimates of an observable are
averaged; their mean minus the exact value is the bias, their spread the
variance of one weighted estimate.  Errors come from the jackknife or the
bootstrap over the groups; the bias is then fitted by a M^-b (least squares
in log|bias| weighted by the errors) and, along beta at fixed M, by
a + b / beta.  RMSD = sqrt(bias^2 + variance) (Eq. (RMSD)).  Wang et al.'s
estimate of the free-energy bias, (beta / 2) var F-hat, is given per spin.

Exact references for the periodic ferromagnet come from its density of
states (``pa_exact_dos``): ln Z, e, c and f per spin.

Everything here is host-side statistics over a few thousand numbers; the
weighted averages themselves are computed on the device.
"""
from __future__ import annotations

import math

import numpy as np


def exact_fm(g, L, beta):
    """ln Z, e, c, f per spin of the periodic L x L ferromagnet at beta from
    its density of states g[m] (E = -2N + 4m)."""
    N = L * L
    E = np.array([-2 * N + 4 * m for m in range(N + 1)], np.float64)
    lng = np.array([math.log(x) if x > 0 else -np.inf for x in g], np.float64)
    a = lng - beta * E
    top = a.max()
    w = np.exp(a - top)
    Z = w.sum()
    lnZ = top + math.log(Z)
    p = w / Z
    mean = (p * E).sum()
    var = (p * (E - mean) ** 2).sum()
    out = {"lnZ": lnZ, "e": mean / N, "c": beta * beta * var / N}
    out["f"] = -lnZ / (beta * N) if beta > 0 else float("nan")
    return out


def jackknife(samples, stat=np.mean):
    """Delete-one jackknife over the first axis: (estimate, standard error)."""
    x = np.asarray(samples, np.float64)
    n = x.shape[0]
    full = stat(x, axis=0)
    loo = np.stack([stat(np.delete(x, k, axis=0), axis=0) for k in range(n)])
    err = np.sqrt((n - 1) / n * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))
    return full, err


def bootstrap(samples, stat=np.mean, n_boot=2000, seed=0):
    """Bootstrap over the first axis: (estimate, standard deviation of the
    resampled statistic)."""
    x = np.asarray(samples, np.float64)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    reps = np.stack([stat(x[rng.integers(0, n, n)], axis=0) for _ in range(n_boot)])
    return stat(x, axis=0), reps.std(axis=0)


def fit_power_law(M, y, sigma):
    """Least-squares fit of y = a M^-b: a straight line in (ln M, ln y) with
    weights 1 / (sigma / y)^2.  Returns (a, b, sigma_b), sigma_b the
    standard fit error."""
    M = np.asarray(M, np.float64)
    y = np.asarray(y, np.float64)
    s = np.asarray(sigma, np.float64) / y
    x, z, w = np.log(M), np.log(y), 1.0 / s ** 2
    S, Sx, Sz = w.sum(), (w * x).sum(), (w * z).sum()
    Sxx, Sxz = (w * x * x).sum(), (w * x * z).sum()
    det = S * Sxx - Sx * Sx
    slope = (S * Sxz - Sx * Sz) / det
    icpt = (Sxx * Sz - Sx * Sxz) / det
    return math.exp(icpt), -slope, math.sqrt(S / det)


def fit_a_plus_b_over_beta(beta, y):
    """Ordinary least squares of y = a + b / beta: (a, b)."""
    x = 1.0 / np.asarray(beta, np.float64)
    y = np.asarray(y, np.float64)
    n = len(x)
    det = n * (x * x).sum() - x.sum() ** 2
    b = (n * (x * y).sum() - x.sum() * y.sum()) / det
    a = (y.sum() - b * x.sum()) / n
    return a, b


def rmsd(bias, variance):
    """Eq. (RMSD): sqrt(bias^2 + variance)."""
    return np.sqrt(np.asarray(bias) ** 2 + np.asarray(variance))


def wang_f_bias(beta, var_f, N):
    """Wang et al.'s large-R bias of the free energy, (beta / 2) var F-hat,
    per spin: with F = N f, (beta / 2) N^2 var f-hat / N = beta N var f-hat / 2."""
    return beta * N * np.asarray(var_f) / 2.0


def weighted_f(wavg, beta, N):
    """f per spin of each group's weighted free energy, -(-beta W[F]) / (beta N)."""
    return -np.asarray(wavg["minus_beta_WF"]) / (np.asarray(beta) * N)
