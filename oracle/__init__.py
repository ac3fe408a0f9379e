"""ctypes binding of the CPU oracle (oracle/pa_oracle.c).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library; the only common input is the plain run descriptor
built by ``workloads.py``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, ERR_ARG, ERR_CAPACITY, ERR_STATE, ERR_NUMERIC = 0, 1, 3, 4, 5


class _Desc(C.Structure):
    _fields_ = [("L", C.c_int32), ("model", C.c_int32), ("seed", C.c_uint64),
                ("disorder_seed", C.c_uint64), ("R", C.c_int32), ("R_cap", C.c_int32),
                ("theta", C.c_int32), ("K", C.c_int32), ("beta", C.POINTER(C.c_double)),
                ("resampling", C.c_int32), ("overlap", C.c_int32), ("qhist", C.c_int32)]


OBS_FIELDS = [("R_i", np.int64), ("lnQ", np.float64), ("A", np.float64),
              ("sumE", np.int64), ("sumE2", np.int64), ("sumAbsM", np.int64),
              ("sumM2", np.int64), ("nPairs", np.int64), ("sumQ", np.int64),
              ("sumAbsQ", np.int64), ("sumQ2", np.int64), ("sumQl", np.int64),
              ("sumQl2", np.int64), ("famSumSq", np.int64), ("famMax", np.int64),
              ("nFam", np.int64), ("Emin", np.int32), ("status", np.int32)]
OBS_DTYPE = np.dtype(OBS_FIELDS)

WAVG_FIELDS = [(n, np.float64) for n in
               ("W_e", "W_e2", "Wvar_c", "Wconf_c", "W_m", "W_m2", "Wvar_chi", "Wconf_chi",
                "W_absq", "W_q2", "W_ql", "minus_beta_WF", "var_w", "var_w_pred")] + \
              [("n_included", np.int32), ("_pad", np.int32)]
WAVG_DTYPE = np.dtype(WAVG_FIELDS)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.or_create.restype = vp
        L.or_create.argtypes = [C.POINTER(_Desc)]
        L.or_destroy.argtypes = [vp]
        for name in ("or_anneal_step", "or_resample", "or_sweep", "or_measure"):
            getattr(L, name).argtypes = [vp, C.c_int]
            getattr(L, name).restype = C.c_int
        L.or_anneal_all.argtypes = [vp]
        L.or_get_info.argtypes = [vp, vp]
        L.or_energy_mismatches.argtypes = [vp]
        L.or_energy_mismatches.restype = C.c_int64
        L.or_get_state.argtypes = [vp, C.c_int, vp, vp, vp, vp]
        L.or_get_state.restype = C.c_int32
        L.or_get_counts.argtypes = [vp, C.c_int, vp, vp, vp]
        L.or_get_counts.restype = C.c_int32
        L.or_get_couplings.argtypes = [vp, vp, vp]
        L.or_get_obs.argtypes = [vp, vp]
        L.or_get_qhist.argtypes = [vp, vp]
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_philox4x32_10.restype = None
        L.or_sweep_threshold.argtypes = [C.c_double, C.c_int]
        L.or_sweep_threshold.restype = C.c_uint64
        L.or_reweight_x.argtypes = [C.c_double, C.c_int]
        L.or_reweight_x.restype = C.c_double
        L.or_reweight_X.argtypes = [C.c_double, C.c_int]
        L.or_reweight_X.restype = C.c_uint64
        L.or_sweep_draw.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_sweep_draw.restype = C.c_uint32
        L.or_set_dos.argtypes = [vp, vp]
        L.or_set_dos.restype = C.c_int
        L.or_exact_dos.argtypes = [C.c_int, vp]
        L.or_exact_dos.restype = C.c_int
        L.or_random_permutation.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int, vp]
        L.or_random_permutation.restype = C.c_int
        L.or_wang_repair.argtypes = [vp, C.c_int, vp, vp]
        L.or_wang_repair.restype = C.c_int
        L.or_get_pairing.argtypes = [vp, C.c_int, vp]
        L.or_get_pairing.restype = C.c_int
        L.or_weighted_average.argtypes = [vp, vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]
        L.or_log_weights.argtypes = [vp, C.c_int, C.c_int, vp, C.c_int, vp]
        L.or_weighted_qhist.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp]
        L.or_family_stats.argtypes = [vp, vp, vp, C.c_int, vp]
        L.or_get_rho.argtypes = [vp, vp]
        L.or_many_runs.argtypes = [C.POINTER(_Desc), C.c_int, vp, vp, vp]
        L.or_many_runs_obs.argtypes = [C.POINTER(_Desc), C.c_int, vp]
        L.or_sweep_groups.argtypes = [vp, C.c_int, vp, C.c_int]
        L.or_sweep_groups.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _mkdesc(d: dict):
    beta = np.ascontiguousarray(d["beta"], dtype=np.float64)
    cd = _Desc(L=d["L"], model=d["model"], seed=d["seed"], disorder_seed=d["disorder_seed"],
               R=d["R"], R_cap=d["R_cap"], theta=d["theta"], K=len(beta),
               beta=beta.ctypes.data_as(C.POINTER(C.c_double)),
               resampling=d["resampling"], overlap=d["overlap"], qhist=d.get("qhist", 0))
    return cd, beta


class OracleRun:
    """One PA run on the CPU oracle; method names follow the paper's steps."""

    def __init__(self, desc: dict):
        self.desc = dict(desc)
        self._cd, self._beta = _mkdesc(desc)
        self._h = lib().or_create(C.byref(self._cd))
        if not self._h:
            raise ValueError("oracle rejected the run descriptor")
        info = np.zeros(6, np.int32)
        lib().or_get_info(self._h, _ptr(info))
        self.N, self.npop, self.K = int(info[2]), int(info[3]), int(info[4])
        if desc["theta"] == -1 and desc["L"] > 8:
            # theta = infinity beyond the C transfer matrix's range: the
            # density of states of the product formula (oracle/dos.py)
            from .dos import fm_dos_doubles
            gd = np.ascontiguousarray(fm_dos_doubles(desc["L"]), dtype=np.float64)
            if lib().or_set_dos(self._h, _ptr(gd)) != OK:
                raise ValueError("oracle rejected the density of states")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    @property
    def i(self):
        info = np.zeros(6, np.int32)
        lib().or_get_info(self._h, _ptr(info))
        return int(info[0])

    def anneal_step(self, i):
        return lib().or_anneal_step(self._h, i)

    def resample(self, i):
        return lib().or_resample(self._h, i)

    def sweep(self, i):
        return lib().or_sweep(self._h, i)

    def measure(self, i):
        return lib().or_measure(self._h, i)

    def sweep_groups(self, i, groups):
        """Step (iv) for the listed 64-replica groups only (sampling of large
        configurations; the run cannot be continued afterwards)."""
        g = np.ascontiguousarray(groups, dtype=np.int32)
        return lib().or_sweep_groups(self._h, i, _ptr(g), len(g))

    def step(self, i):
        for f in (self.anneal_step, self.resample, self.sweep, self.measure):
            st = f(i)
            if st:
                raise RuntimeError(f"oracle step {i} failed with status {st}")

    def run_all(self):
        st = lib().or_anneal_all(self._h)
        if st:
            raise RuntimeError(f"oracle run failed with status {st}")
        return self

    def energy_mismatches(self):
        return int(lib().or_energy_mismatches(self._h))

    def state(self, pop=0):
        """(spins [R_i, N] int8 +-1, E [R_i] int32, fam [R_i] int32, status)."""
        Rc = self.desc["R_cap"]
        s = np.zeros((Rc, self.N), np.int8)
        E = np.zeros(Rc, np.int32)
        f = np.zeros(Rc, np.int32)
        st = np.zeros(1, np.int32)
        Ri = lib().or_get_state(self._h, pop, _ptr(s), _ptr(E), _ptr(f), _ptr(st))
        return s[:Ri].copy(), E[:Ri].copy(), f[:Ri].copy(), int(st[0])

    def counts(self, pop=0):
        """(r [R_{i-1}], X [R_{i-1}], S_X) of the last resampling."""
        Rc = self.desc["R_cap"]
        r = np.zeros(Rc, np.int32)
        X = np.zeros(Rc, np.uint64)
        SX = np.zeros(1, np.uint64)
        Rp = lib().or_get_counts(self._h, pop, _ptr(r), _ptr(X), _ptr(SX))
        return r[:Rp].copy(), X[:Rp].copy(), int(SX[0])

    def couplings(self):
        jR = np.zeros(self.N, np.int8)
        jD = np.zeros(self.N, np.int8)
        lib().or_get_couplings(self._h, _ptr(jR), _ptr(jD))
        return jR, jD

    def obs(self):
        """Structured array [npop, K] of per-temperature records."""
        out = np.zeros((self.npop, self.K), OBS_DTYPE)
        lib().or_get_obs(self._h, _ptr(out))
        return out

    def pairing(self, pop=0):
        """(status, pairs) of the permutation pairing at the current
        temperature: pairs[k] is the partner of replica k."""
        _, _, fam, _ = self.state(pop)
        out = np.zeros(max(len(fam), 1), np.int32)
        st = lib().or_get_pairing(self._h, pop, _ptr(out))
        return st, out[:len(fam)]

    def rho(self):
        """Mean square family size rho_t [npop, K] (Eq. (rho_t)), computed in
        the measurement from the family histogram."""
        out = np.zeros((self.npop, self.K), np.float64)
        lib().or_get_rho(self._h, _ptr(out))
        return out

    def qhist(self):
        out = np.zeros((self.npop, self.K, self.N + 1), np.int32)
        if lib().or_get_qhist(self._h, _ptr(out)):
            raise ValueError("run was created without overlap histograms")
        return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sweep_threshold(beta, dE):
    return int(lib().or_sweep_threshold(float(beta), int(dE)))


def reweight_x(dbeta, k):
    return float(lib().or_reweight_x(float(dbeta), int(k)))


def reweight_X(dbeta, k):
    return int(lib().or_reweight_X(float(dbeta), int(k)))


def sweep_draw(seed, n, j, i, pop, s):
    return int(lib().or_sweep_draw(seed, n, j, i, pop, s))


FAMSTAT_DTYPE = np.dtype([("rho_t", np.float64), ("R_i", np.int32), ("famMax", np.int32),
                          ("large", np.int32), ("excluded", np.int32)])

EXCLUDE_LARGE_FAMILY = 2   # flag OR-ed into `kind`


def exact_dos(L):
    """Exact density of states of the periodic L x L ferromagnet (L <= 8):
    g[m] = number of configurations with E = -2N + 4m, as Python ints."""
    N = L * L
    raw = np.zeros(2 * (N + 1), np.uint64)
    st = lib().or_exact_dos(L, _ptr(raw))
    assert st == OK, st
    return [int(raw[2 * m]) | (int(raw[2 * m + 1]) << 64) for m in range(N + 1)]


def random_permutation(seed, i, pop, R, which=0):
    """Permutation of [0, R) drawn for the pairing at temperature i
    (which = 0: the initial pi, 1: the search pattern sigma)."""
    out = np.zeros(max(R, 1), np.int32)
    st = lib().or_random_permutation(C.c_uint64(seed), i, pop, R, which, _ptr(out))
    assert st == OK, st
    return out[:R]


def wang_repair(fam, pi, sigma=None):
    """Permutation pairing without incestuous pairs (Sec. III D): returns
    (status, repaired pi); status 1 when a family exceeds R/2 (pi unchanged)."""
    fam = np.ascontiguousarray(fam, np.int32)
    out = np.ascontiguousarray(pi, np.int32).copy()
    sg = None if sigma is None else np.ascontiguousarray(sigma, np.int32)
    st = lib().or_wang_repair(_ptr(fam), len(fam), _ptr(out), None if sg is None else _ptr(sg))
    return st, out


def weighted_average(obs_mk, beta, N, R, kind=0, obs_other=None):
    """obs_mk: structured [M, K] records (one population per run); obs_other:
    the other population's records of two-population runs (for the
    large-family exclusion), or None."""
    obs_mk = np.ascontiguousarray(obs_mk, dtype=OBS_DTYPE)
    M, K = obs_mk.shape
    other = None if obs_other is None else np.ascontiguousarray(obs_other, dtype=OBS_DTYPE)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.int32), (M,)), dtype=np.int32)
    out = np.zeros(K, WAVG_DTYPE)
    st = lib().or_weighted_average(_ptr(obs_mk), _ptr(other), M, K, _ptr(beta), int(N), _ptr(R), int(kind),
                                   _ptr(out))
    if st:
        raise ValueError(f"or_weighted_average failed: {st}")
    return out


def log_weights(obs_mk, R, kind=0):
    """The oracle's log free-energy weights a[m, i] of M runs (full weight,
    kind 0, Eq. (appropriateWeight); simplified, kind 1, Eq. (simpleWeight));
    NaN where a record's status is not OK."""
    obs_mk = np.ascontiguousarray(obs_mk, dtype=OBS_DTYPE)
    M, K = obs_mk.shape
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.int32), (M,)), dtype=np.int32)
    out = np.zeros((M, K), np.float64)
    st = lib().or_log_weights(_ptr(obs_mk), M, K, _ptr(R), int(kind), _ptr(out))
    if st:
        raise ValueError(f"or_log_weights failed: {st}")
    return out


def weighted_qhist(obs_mk, qh_mkd, N, R, kind=0, obs_other=None):
    """Eq. (W_conf_q) for one group: obs_mk [M, K] records and qh_mkd
    [M, K, N+1] histograms of the weighted population; returns [K, N+1]."""
    obs_mk = np.ascontiguousarray(obs_mk, dtype=OBS_DTYPE)
    M, K = obs_mk.shape
    other = None if obs_other is None else np.ascontiguousarray(obs_other, dtype=OBS_DTYPE)
    qh = np.ascontiguousarray(qh_mkd, dtype=np.int32)
    assert qh.shape == (M, K, N + 1)
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.int32), (M,)), dtype=np.int32)
    out = np.zeros((K, N + 1), np.float64)
    st = lib().or_weighted_qhist(_ptr(obs_mk), _ptr(other), _ptr(qh), M, K, int(N), _ptr(R), int(kind), _ptr(out))
    if st:
        raise ValueError(f"or_weighted_qhist failed: {st}")
    return out


def family_stats(rho_k, obs_k, obs_other_k=None):
    """Family statistics [K] of one run's population: rho_t (Eq. (rho_t),
    from OracleRun.rho()), largest family, > R_i/2 flag, exclusion flag."""
    obs_k = np.ascontiguousarray(obs_k, dtype=OBS_DTYPE)
    K = obs_k.shape[0]
    rho = np.ascontiguousarray(rho_k, dtype=np.float64)
    other = None if obs_other_k is None else np.ascontiguousarray(obs_other_k, dtype=OBS_DTYPE)
    out = np.zeros(K, FAMSTAT_DTYPE)
    lib().or_family_stats(_ptr(rho), _ptr(obs_k), _ptr(other), K, _ptr(out))
    return out


def many_runs(desc: dict, M: int):
    """A [M,K], sumE [M,K], R_i [M,K] of M runs with seeds seed+m."""
    cd, beta = _mkdesc(desc)
    K = len(beta)
    A = np.zeros((M, K), np.float64)
    sE = np.zeros((M, K), np.int64)
    Rr = np.zeros((M, K), np.int64)
    st = lib().or_many_runs(C.byref(cd), M, _ptr(A), _ptr(sE), _ptr(Rr))
    if st:
        raise RuntimeError(f"or_many_runs failed: {st}")
    return A, sE, Rr


def many_runs_obs(desc: dict, M: int):
    """Records [M, K] (population 0) of M runs with seeds seed+m."""
    cd, beta = _mkdesc(desc)
    out = np.zeros((M, len(beta)), OBS_DTYPE)
    st = lib().or_many_runs_obs(C.byref(cd), M, _ptr(out))
    if st:
        raise RuntimeError(f"or_many_runs_obs failed: {st}")
    return out
