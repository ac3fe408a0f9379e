"""Exact equilibrium references for small 2D Ising systems (test pins).

Independent of both the oracle and the GPU library: everything here is a
textbook method written from its mathematical definition.

* ``enumerate_states`` -- brute force over all 2^N configurations (N <= 16),
  for the ferromagnet or any coupling set (+-J spin glass).
* ``fm_transfer_lnZ`` -- row-to-row transfer matrix of the periodic L x L
  ferromagnet, Z = Tr T^L (L <= 10).
* ``fm_transfer_M_distribution`` -- the same transfer matrix with a complex
  "field" that counts up spins, inverted by a discrete Fourier transform to
  give the exact weight of every magnetisation (L <= 8).
* ``kaufman_lnZ`` -- Kaufman's closed form for the partition function of the
  finite periodic L x L ferromagnet (Phys. Rev. 76, 1232 (1949)), in mpmath,
  with e and c by numerical differentiation of ln Z.  The paper quotes exact
  finite-L results as its reference solution (Sec. V A 3); the formula is
  written from the published mathematics and checked here against brute force
  and the transfer matrix before use.

Conventions follow the paper: H = -sum_<mn> J_mn s_m s_n over the 2N bonds of
the periodic lattice (Eqs. (H_FM), (H_EA)), Z(beta) = sum exp(-beta H).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# --------------------------------------------------------------- brute force

def _bonds(L):
    """Bond list [(n, m)] with m = right(n) then m = down(n), n = y*L + x."""
    out = []
    for n in range(L * L):
        x, y = n % L, n // L
        out.append((n, y * L + (x + 1) % L))
        out.append((n, ((y + 1) % L) * L + x))
    return out


def all_configs(N):
    """All 2^N configurations as an int8 array [2^N, N] of +-1 (bit n of the
    index set means s_n = -1)."""
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)


def enumerate_states(L, jR=None, jD=None):
    """Energies and magnetisations of all configurations of the L x L torus.

    jR[n], jD[n] are the couplings of bonds (n, right(n)) and (n, down(n));
    None means the ferromagnet (all +1).  Returns (S [2^N,N], E [2^N], M [2^N]).
    """
    N = L * L
    if N > 16:
        raise ValueError("brute force limited to N <= 16")
    S = all_configs(N).astype(np.int32)
    jR = np.ones(N, np.int32) if jR is None else np.asarray(jR, np.int32)
    jD = np.ones(N, np.int32) if jD is None else np.asarray(jD, np.int32)
    E = np.zeros(2 ** N, np.int64)
    for n in range(N):
        x, y = n % L, n // L
        r = y * L + (x + 1) % L
        d = ((y + 1) % L) * L + x
        E -= jR[n] * S[:, n] * S[:, r]
        E -= jD[n] * S[:, n] * S[:, d]
    M = S.sum(axis=1).astype(np.int64)
    return S, E, M


def boltzmann(E, beta):
    w = np.exp(-beta * (E - E.min()))
    return w / w.sum()


def exact_from_enumeration(E, M, beta, N):
    """ln Z, e, c, <|m|>, <m^2> per spin at beta from an enumeration."""
    E = np.asarray(E, np.float64)
    a = -beta * E
    amax = a.max()
    lnZ = amax + math.log(np.exp(a - amax).sum())
    p = np.exp(a - lnZ)
    e = (p * E).sum() / N
    e2 = (p * E * E).sum() / N ** 2
    c = beta ** 2 * N * (e2 - e * e)
    m = (p * np.abs(M)).sum() / N
    m2 = (p * M.astype(np.float64) ** 2).sum() / N ** 2
    return dict(lnZ=lnZ, e=e, c=c, m=m, m2=m2, chi=beta * N * (m2 - m * m))


def overlap_distributions(S, E, L, beta, jR=None, jD=None):
    """Exact P(q) and P(q_l) of two independent replicas at beta.

    q = (1/N) sum_n s_n s'_n and q_l = (1/2N) sum_bonds (s_m s_n)(s'_m s'_n).
    Both depend only on z = s * s' (elementwise), so the joint law follows
    from the autocorrelation h(z) = sum_x pi(x) pi(x*z), computed with a
    Walsh-Hadamard transform over the 2^N states.
    Returns (P_q indexed by Hamming distance 0..N, dict q_l value -> prob).
    """
    N = L * L
    pi = boltzmann(E, beta)
    # index of configuration: bit n set <=> s_n = -1, so x*z <-> index xor
    h = _xor_autocorrelation(pi)
    idx = np.arange(2 ** N)
    ham = np.array([bin(i).count("1") for i in idx])
    Pq = np.bincount(ham, weights=h, minlength=N + 1)
    Z = all_configs(N).astype(np.int32)
    ql = np.zeros(2 ** N, np.int64)
    for (n, m) in _bonds(L):
        ql += Z[:, n] * Z[:, m]
    Pql = {}
    for v, w in zip(ql, h):
        Pql[int(v)] = Pql.get(int(v), 0.0) + w
    return Pq, Pql


def _xor_autocorrelation(pi):
    """h(z) = sum_x pi(x) pi(x xor z) via the Walsh-Hadamard transform."""
    f = _fwht(pi.astype(np.float64).copy())
    return _fwht(f * f) / len(pi)


def _fwht(a):
    n = len(a)
    h = 1
    while h < n:
        a = a.reshape(-1, 2 * h)
        x = a[:, :h].copy()
        y = a[:, h:].copy()
        a[:, :h] = x + y
        a[:, h:] = x - y
        a = a.reshape(-1)
        h *= 2
    return a


# ---------------------------------------------------------- transfer matrix

def _row_tables(L):
    rows = all_configs(L).astype(np.int64)              # [2^L, L]
    e_in = -(rows * np.roll(rows, -1, axis=1)).sum(1)   # bonds inside a row
    e_ab = -(rows @ rows.T)                             # vertical bonds a -> b
    up = (rows > 0).sum(1)
    return rows, e_in, e_ab, up


def fm_transfer_lnZ(L, beta):
    """ln Z of the periodic L x L ferromagnet, Z = Tr T^L (exact)."""
    _, e_in, e_ab, _ = _row_tables(L)
    expo = -beta * (0.5 * e_in[:, None] + e_ab + 0.5 * e_in[None, :])
    shift = expo.max()
    T = np.exp(expo - shift)
    lam = np.linalg.eigvalsh(T)
    lmax = np.abs(lam).max()
    return L * shift + L * math.log(lmax) + math.log(((lam / lmax) ** L).sum())


def fm_transfer_M_distribution(L, beta):
    """Exact probabilities of M = 2*(#up) - N for the L x L ferromagnet.

    Z_k = Tr (T D_k)^L with D_k = diag(w^(k up(b))), w = exp(2 pi i/(N+1)),
    equals sum_u g(u) w^(k u); the inverse DFT recovers g(u).
    Returns (M values [N+1], probabilities [N+1]).
    """
    N = L * L
    _, e_in, e_ab, up = _row_tables(L)
    expo = -beta * (0.5 * e_in[:, None] + e_ab + 0.5 * e_in[None, :])
    T = np.exp(expo - expo.max())
    lmax = np.abs(np.linalg.eigvalsh(T)).max()
    T = T / lmax
    Zk = np.zeros(N + 1, np.complex128)
    for k in range(N + 1):
        w = np.exp(2j * np.pi * k * up / (N + 1))
        Tk = T * w[None, :]
        lam = np.linalg.eigvals(Tk)
        Zk[k] = (lam ** L).sum()
    g = np.fft.fft(Zk).real / (N + 1)        # g(u) = (1/(N+1)) sum_k Z_k w^{-k u}
    g = np.clip(g, 0.0, None)
    p = g / g.sum()
    Mv = 2 * np.arange(N + 1) - N
    return Mv, p


# ------------------------------------------------------------------ Kaufman

def kaufman_lnZ(L, beta, dps=40):
    """ln Z of the periodic L x L ferromagnet (J = 1) by Kaufman's formula.

    Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4), K = beta,
    Z1 = prod_{r=0}^{L-1} 2 cosh(L g_{2r+1}/2), Z2 = prod 2 sinh(L g_{2r+1}/2),
    Z3 = prod_{r=0}^{L-1} 2 cosh(L g_{2r}/2),   Z4 = prod 2 sinh(L g_{2r}/2),
    cosh g_k = cosh 2K coth 2K - cos(pi k / L) for k >= 1 (g_k > 0), and
    g_0 = 2K + ln tanh K, which is negative above the critical temperature.
    """
    import mpmath as mp
    with mp.workdps(max(dps, mp.mp.dps)):
        K = mp.mpf(beta)
        if K == 0:
            return mp.mpf(L * L) * mp.log(2)
        N = L * L
        ch = mp.cosh(2 * K) / mp.tanh(2 * K)

        def g(k):
            if k == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(ch - mp.cos(mp.pi * k / L))

        odd = [g(2 * r + 1) for r in range(L)]
        even = [g(2 * r) for r in range(L)]
        Z1 = mp.fprod(2 * mp.cosh(L * x / 2) for x in odd)
        Z2 = mp.fprod(2 * mp.sinh(L * x / 2) for x in odd)
        Z3 = mp.fprod(2 * mp.cosh(L * x / 2) for x in even)
        Z4 = mp.fprod(2 * mp.sinh(L * x / 2) for x in even)
        pref = mp.mpf(1) / 2 * (2 * mp.sinh(2 * K)) ** (mp.mpf(N) / 2)
        return mp.log(pref * (Z1 + Z2 + Z3 + Z4))


def kaufman_thermo(L, beta, dps=40):
    """(lnZ, e, c) per the Kaufman formula; e = -(1/N) d lnZ/d beta,
    c = (beta^2/N) d^2 lnZ/d beta^2, derivatives by mpmath."""
    import mpmath as mp
    N = L * L
    with mp.workdps(dps):
        f = lambda b: kaufman_lnZ(L, b, dps=dps)
        lnZ = f(beta)
        d1 = mp.diff(f, mp.mpf(beta), 1)
        d2 = mp.diff(f, mp.mpf(beta), 2)
        return float(lnZ), float(-d1 / N), float(mp.mpf(beta) ** 2 * d2 / N)


BETA_C = 0.5 * math.log(1.0 + math.sqrt(2.0))
