"""Exact density of states of the periodic L x L Ising ferromagnet.

TEST INFRASTRUCTURE (part of the oracle: only tests/, the smoke check and
the CPU-baseline leg of the benchmark use it).

The theta = infinity limit of Sec. V C samples energies from the exact
distribution g(E) exp(-beta E) / Z; the paper takes g from Beale's exact
evaluation of the finite-lattice partition function.  Here g is written
out from Kaufman's closed form for the torus, as a polynomial in
y = exp(-2 beta) (Beale's observation that its coefficients are the exact
integer counts):

    sum_u g_u y^u = (1/2) (Q_00 + Q_01 + Q_10 + Q_11),

u the number of unsatisfied bonds (E = -2N + 2u), where Q_ab is the product,
over the momenta p = 2 pi (k + a/2) / L, q = 2 pi (l + b/2) / L
(k, l = 0 .. L-1) taken once per pair {(p, q), (-p, -q)}, of

    f_pq(y) = (1 + y^2)^2 - 2 y (1 - y^2) (cos p + cos q),

and for the momenta equal to their own negatives (p, q in {0, pi}, only
in Q_00 for even L) of the square roots (1 - 2y - y^2) (p = q = 0),
(1 + 2y - y^2) (p = q = pi) and (1 + y^2) (p != q).  The square of that
product is the product of f_pq over all momenta, the Kac-Ward / Kasteleyn
determinant of the torus with the boundary condition (a, b).

The product is evaluated in mpmath with enough digits that every
coefficient (at most 12^(N/2) in magnitude) rounds to its exact integer.
This module shares nothing with the library; the pins are in
tests/test_oracle_dos.py (enumeration and the transfer matrix at L <= 8,
Kaufman's partition function at larger L, sum 2^N, symmetry).
"""
from __future__ import annotations

import functools

import mpmath as mp


def _polymul(a, b):
    out = [mp.mpf(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _Q(L, a, b):
    """Q_ab as a list of mpf coefficients of y^0 .. y^(2N)."""
    one = mp.mpf(1)
    # momentum of index k with offset a: p = pi (2k + a) / L; negation maps
    # 2k + a to 2L - 2k - a (mod 2L)
    idx = lambda k, s: (2 * k + s) % (2 * L)   # noqa: E731
    neg = lambda j: (-j) % (2 * L)             # noqa: E731
    cosv = {j: mp.cos(mp.pi * j / L) for j in range(2 * L)}
    P = [one]
    done = set()
    for k in range(L):
        for l in range(L):
            jp, jq = idx(k, a), idx(l, b)
            if (jp, jq) in done:
                continue
            partner = (neg(jp), neg(jq))
            done.add((jp, jq))
            if partner == (jp, jq):                  # p, q in {0, pi}
                cp, cq = int(mp.nint(cosv[jp])), int(mp.nint(cosv[jq]))
                if cp == 1 and cq == 1:
                    r = [one, -2 * one, -one]
                elif cp == -1 and cq == -1:
                    r = [one, 2 * one, -one]
                else:
                    r = [one, mp.mpf(0), one]
                P = _polymul(P, r)
                continue
            done.add(partner)
            s = cosv[jp] + cosv[jq]
            P = _polymul(P, [one, -2 * s, 2 * one, 2 * s, one])
    return P


@functools.lru_cache(maxsize=None)
def fm_dos(L: int) -> tuple:
    """g_m = number of configurations of the periodic L x L ferromagnet with
    E = -2N + 4m, m = 0 .. N, as Python ints (L even, 4 <= L <= 30)."""
    if L < 4 or L > 30 or L % 2:
        raise ValueError("L must be even, 4 <= L <= 30")
    N = L * L
    digits = int(0.6 * N) + 60          # 12^(N/2) < 10^(0.54 N)
    with mp.workdps(digits):
        total = [mp.mpf(0)] * (2 * N + 1)
        for a in (0, 1):
            for b in (0, 1):
                for u, c in enumerate(_Q(L, a, b)):
                    total[u] += c
        g_u = [int(mp.nint(c / 2)) for c in total]
    for u in range(1, 2 * N + 1, 2):
        if g_u[u] != 0:
            raise ArithmeticError("odd number of unsatisfied bonds on the torus")
    g = tuple(g_u[2 * m] for m in range(N + 1))
    if sum(g) != 2 ** N or any(x < 0 for x in g):
        raise ArithmeticError("density of states does not count 2^N configurations")
    return g


def fm_dos_doubles(L: int) -> list:
    """g_m rounded to the nearest double (ties to even), as the draw
    thresholds of the theta = infinity limit use them."""
    return [float(x) for x in fm_dos(L)]


def lnZ_from_dos(L: int, beta: float, dps: int = 40):
    """ln Z(beta) = ln sum_m g_m exp(-beta (-2N + 4m)), in mpmath."""
    N = L * L
    g = fm_dos(L)
    with mp.workdps(dps):
        b = mp.mpf(beta)
        return mp.log(mp.fsum(mp.mpf(x) * mp.exp(-b * (-2 * N + 4 * m)) for m, x in enumerate(g)))


__all__ = ["fm_dos", "fm_dos_doubles", "lnZ_from_dos"]
