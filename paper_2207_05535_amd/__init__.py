"""MI355X population annealing with weighted averaging -- Python binding.

A thin ctypes layer over ``libpa.so`` (the C ABI of ``include/pa.h``): the
functions below carry the ABI's names and only marshal arguments.  Every step
of the algorithm runs in the library's HIP kernels; PyTorch is used only to
allocate the device workspace and to supply the stream.  If the library has
not been built, importing works but every call raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa.so")

PA_OK, PA_ERR_ARG, PA_ERR_NOMEM, PA_ERR_CAPACITY, PA_ERR_STATE, PA_ERR_NUMERIC, PA_ERR_DEVICE = range(7)
PA_FM, PA_EA_PMJ = 0, 1
PA_MULTINOMIAL, PA_NEAREST_INT = 0, 1
PA_INT8, PA_MSC64 = 0, 1
PA_Q_NONE, PA_Q_INDEX_SHIFT, PA_Q_TWO_POP, PA_Q_WANG, PA_Q_WANG_RDM = 0, 1, 2, 3, 4
PA_W_FULL, PA_W_SIMPLE = 0, 1
PA_W_EXCLUDE_LARGE_FAMILY = 2   # flag OR-ed into a weight kind
PA_THETA_EXACT = -1             # theta = infinity: energies drawn from the exact distribution
PA_STATIC_WORKSPACE_BYTES = 128 << 20   # the device array pa_create_static uses

REPRS = {"int8": PA_INT8, "msc": PA_MSC64, PA_INT8: PA_INT8, PA_MSC64: PA_MSC64}


class pa_run_desc(C.Structure):
    _fields_ = [("L", C.c_int32), ("model", C.c_int32), ("seed", C.c_uint64),
                ("disorder_seed", C.c_uint64), ("R", C.c_int32), ("R_cap", C.c_int32),
                ("theta", C.c_int32), ("K", C.c_int32), ("beta", C.POINTER(C.c_double)),
                ("resampling", C.c_int32), ("overlap", C.c_int32), ("qhist", C.c_int32)]


PA_OBS_DTYPE = np.dtype([
    ("R_i", np.int64), ("lnQ", np.float64), ("A", np.float64), ("sumE", np.int64),
    ("sumE2", np.int64), ("sumAbsM", np.int64), ("sumM2", np.int64), ("nPairs", np.int64),
    ("sumQ", np.int64), ("sumAbsQ", np.int64), ("sumQ2", np.int64), ("sumQl", np.int64),
    ("sumQl2", np.int64), ("famSumSq", np.int64), ("famMax", np.int64), ("nFam", np.int64),
    ("Emin", np.int32), ("status", np.int32)])

PA_WAVG_DTYPE = np.dtype(
    [(n, np.float64) for n in ("W_e", "W_e2", "Wvar_c", "Wconf_c", "W_m", "W_m2", "Wvar_chi",
                               "Wconf_chi", "W_absq", "W_q2", "W_ql", "minus_beta_WF", "var_w",
                               "var_w_pred")] + [("n_included", np.int32), ("_pad", np.int32)])


PA_FAMSTAT_DTYPE = np.dtype([("rho_t", np.float64), ("R_i", np.int32), ("famMax", np.int32),
                             ("large", np.int32), ("excluded", np.int32)])


class PAError(RuntimeError):
    def __init__(self, call, status):
        super().__init__(f"{call} failed: {status_str(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """The loaded libpa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        sig = {
            "pa_workspace_size": [vp, i32, i32, vp],
            "pa_create": [vp, i32, i32, vp, C.c_size_t, vp, vp],
            "pa_create_static": [vp, i32, i32, vp, vp],
            "pa_anneal_step": [vp, i32],
            "pa_resample": [vp, i32],
            "pa_sweep": [vp, i32],
            "pa_measure": [vp, i32, vp],
            "pa_run": [vp, i32, i32],
            "pa_weighted_average": [vp, i32, i32, i32, vp],
            "pa_weighted_qhist": [vp, i32, i32, i32, vp],
            "pa_family_stats": [vp, i32, vp],
            "pa_read_obs": [vp, vp],
            "pa_read_qhist": [vp, i32, vp],
            "pa_read_state": [vp, i32, i32, vp, vp, vp, vp, vp, vp],
            "pa_read_pairing": [vp, i32, vp, vp, vp],
            "pa_exact_dos": [i32, vp],
            "pa_exact_dos_wide": [i32, i32, vp],
            "pa_calibrate_philox": [vp, i32, vp],
            "pa_checkpoint": [vp, vp, vp],
            "pa_restore": [vp, vp, C.c_size_t],
            "pa_set_tuning": [vp, i32, i32, i32, i32],
            "pa_set_persistent": [vp, i32],
            "pa_get_tuning": [vp, i32, vp, vp, vp, vp, vp],
            "pa_set_pooled": [vp, i32],
            "pa_set_sweep_chunks": [vp, i32],
            "pa_get_sweep_chunks": [vp, vp],
            "pa_get_sweep_launches": [vp, vp],
            "pa_autotune": [vp, i32, C.c_char_p, vp, vp],
            "pa_read_stats": [vp, vp],
            "pa_destroy": [vp],
            "pa_server_footprint": [vp, i32, vp],
            "pa_server_create": [i32, vp, C.c_size_t, i32, C.c_char_p, vp, vp],
            "pa_server_admit": [vp, vp, vp],
            "pa_server_step": [vp, vp, vp],
            "pa_server_progress": [vp, i32, vp],
            "pa_server_read_obs": [vp, i32, vp, i32],
            "pa_server_release": [vp, i32],
            "pa_server_info": [vp, vp, vp, vp],
            "pa_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.pa_status_str.argtypes = [C.c_int]
        L.pa_status_str.restype = C.c_char_p
        L.pa_last_error.argtypes = [vp]
        L.pa_last_error.restype = C.c_char_p
        L.pa_server_last_error.argtypes = [vp]
        L.pa_server_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def status_str(st: int) -> str:
    try:
        return lib().pa_status_str(int(st)).decode()
    except RuntimeError:
        return str(st)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_descs(runs):
    """ctypes array of pa_run_desc from plain descriptor dicts; returns
    (array, keep-alive list of the schedule arrays)."""
    arr = (pa_run_desc * len(runs))()
    keep = []
    for k, d in enumerate(runs):
        beta = np.ascontiguousarray(d["beta"], dtype=np.float64)
        keep.append(beta)
        arr[k] = pa_run_desc(L=d["L"], model=d["model"], seed=d["seed"],
                             disorder_seed=d["disorder_seed"], R=d["R"], R_cap=d["R_cap"],
                             theta=d["theta"], K=len(beta),
                             beta=beta.ctypes.data_as(C.POINTER(C.c_double)),
                             resampling=d["resampling"], overlap=d["overlap"],
                             qhist=d.get("qhist", 0))
    return arr, keep


# ----------------------------------------------------- C ABI, same names

def pa_workspace_size(runs, repr_) -> int:
    arr, _keep = make_descs(runs)
    n = C.c_size_t(0)
    st = lib().pa_workspace_size(arr, len(runs), REPRS[repr_], C.byref(n))
    if st:
        raise PAError("pa_workspace_size", st)
    return n.value


def pa_create(runs, repr_, dev_ptr: int, nbytes: int, stream_ptr: int):
    arr, _keep = make_descs(runs)
    h = C.c_void_p()
    st = lib().pa_create(arr, len(runs), REPRS[repr_], C.c_void_p(dev_ptr), nbytes,
                         C.c_void_p(stream_ptr), C.byref(h))
    if st:
        raise PAError("pa_create", st)
    return h


def pa_create_static(runs, repr_, stream_ptr: int):
    arr, _keep = make_descs(runs)
    h = C.c_void_p()
    st = lib().pa_create_static(arr, len(runs), REPRS[repr_], C.c_void_p(stream_ptr), C.byref(h))
    if st:
        raise PAError("pa_create_static", st)
    return h


def _chk(call, st, h=None, server=False):
    if st:
        e = PAError(call, st)
        if st == PA_ERR_DEVICE and h is not None:
            text = (lib().pa_server_last_error if server else lib().pa_last_error)(h)
            e.args = (e.args[0] + ": " + text.decode(),)
        raise e


def pa_anneal_step(h, i):
    _chk("pa_anneal_step", lib().pa_anneal_step(h, i), h)


def pa_resample(h, i):
    _chk("pa_resample", lib().pa_resample(h, i), h)


def pa_sweep(h, i):
    _chk("pa_sweep", lib().pa_sweep(h, i), h)


def pa_measure(h, i, out=None):
    _chk("pa_measure", lib().pa_measure(h, i, _p(out)), h)


def pa_run(h, i_begin, i_end):
    _chk("pa_run", lib().pa_run(h, i_begin, i_end), h)


def pa_weighted_average(h, M, kind, pop, out):
    _chk("pa_weighted_average", lib().pa_weighted_average(h, M, kind, pop, _p(out)), h)


def pa_weighted_qhist(h, M, kind, pop, out):
    _chk("pa_weighted_qhist", lib().pa_weighted_qhist(h, M, kind, pop, _p(out)), h)


def pa_family_stats(h, pop, out):
    _chk("pa_family_stats", lib().pa_family_stats(h, pop, _p(out)), h)


def pa_read_obs(h, out):
    _chk("pa_read_obs", lib().pa_read_obs(h, _p(out)), h)


def pa_read_qhist(h, run, out):
    _chk("pa_read_qhist", lib().pa_read_qhist(h, run, _p(out)), h)


def pa_calibrate_philox(calls_per_chain=4096, stream=None):
    """Philox4x32-10 calls per second on the whole device, all in registers
    (two independent chains per lane); 40 VALU instructions per call."""
    out = C.c_double(0.0)
    _chk("pa_calibrate_philox", lib().pa_calibrate_philox(stream, calls_per_chain, C.byref(out)))
    return out.value


def pa_exact_dos(L):
    """Exact density of states of the periodic L x L ferromagnet (even L,
    4 <= L <= 30): g[m] = number of configurations with E = -2N + 4m, as
    Python ints (pa_exact_dos_wide)."""
    N = L * L
    limbs = N // 64 + 1
    raw = np.zeros((N + 1) * limbs, np.uint64)
    _chk("pa_exact_dos_wide", lib().pa_exact_dos_wide(L, limbs, _p(raw)))
    raw = raw.reshape(N + 1, limbs)
    return [sum(int(raw[m, w]) << (64 * w) for w in range(limbs)) for m in range(N + 1)]


def pa_read_pairing(h, run, out):
    st, Ri = C.c_int32(0), C.c_int32(0)
    _chk("pa_read_pairing", lib().pa_read_pairing(h, run, _p(out), C.byref(st), C.byref(Ri)), h)
    return st.value, Ri.value


def pa_read_state(h, run, pop, spins, E, fam, counts):
    Ri, Rp = C.c_int32(0), C.c_int32(0)
    _chk("pa_read_state", lib().pa_read_state(h, run, pop, _p(spins), _p(E), _p(fam), _p(counts),
                                              C.byref(Ri), C.byref(Rp)), h)
    return Ri.value, Rp.value


def pa_checkpoint(h, buf=None):
    n = C.c_size_t(0 if buf is None else len(buf))
    _chk("pa_checkpoint", lib().pa_checkpoint(h, None if buf is None else _p(buf), C.byref(n)), h)
    return n.value


def pa_restore(h, buf):
    _chk("pa_restore", lib().pa_restore(h, _p(buf), len(buf)), h)


def pa_set_tuning(h, L, threads, groups_per_wg, dense_calls=3):
    _chk("pa_set_tuning", lib().pa_set_tuning(h, L, threads, groups_per_wg, dense_calls), h)


def pa_set_persistent(h, on):
    _chk("pa_set_persistent", lib().pa_set_persistent(h, int(on)), h)


def pa_set_pooled(h, on):
    _chk("pa_set_pooled", lib().pa_set_pooled(h, int(on)), h)


def pa_set_sweep_chunks(h, chunks):
    _chk("pa_set_sweep_chunks", lib().pa_set_sweep_chunks(h, int(chunks)), h)


def pa_get_sweep_chunks(h):
    v = C.c_int32(0)
    _chk("pa_get_sweep_chunks", lib().pa_get_sweep_chunks(h, C.byref(v)), h)
    return v.value


def pa_get_sweep_launches(h):
    v = C.c_int32(0)
    _chk("pa_get_sweep_launches", lib().pa_get_sweep_launches(h, C.byref(v)), h)
    return v.value


def pa_get_tuning(h, L):
    v = [C.c_int32(0) for _ in range(5)]
    _chk("pa_get_tuning", lib().pa_get_tuning(h, L, *[C.byref(x) for x in v]), h)
    return dict(threads=v[0].value, groups=v[1].value, dense=v[2].value, persistent=v[3].value,
                pooled=v[4].value)


def pa_autotune(h, steps, cache_path=None):
    tried, rejected = C.c_int32(0), C.c_int32(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _chk("pa_autotune", lib().pa_autotune(h, steps, path, C.byref(tried), C.byref(rejected)), h)
    return dict(tried=tried.value, rejected=rejected.value)


def pa_read_stats(h):
    out = np.zeros(3, np.uint64)
    _chk("pa_read_stats", lib().pa_read_stats(h, _p(out)), h)
    return out


def pa_destroy(h):
    _chk("pa_destroy", lib().pa_destroy(h))


def pa_server_footprint(desc, repr_) -> int:
    arr, _keep = make_descs([desc])
    n = C.c_size_t(0)
    _chk("pa_server_footprint", lib().pa_server_footprint(arr, REPRS[repr_], C.byref(n)))
    return n.value


def pa_server_create(repr_, dev_ptr: int, nbytes: int, max_slots: int, tuning_cache, stream_ptr: int):
    h = C.c_void_p()
    path = None if tuning_cache is None else os.fsencode(tuning_cache)
    _chk("pa_server_create", lib().pa_server_create(REPRS[repr_], C.c_void_p(dev_ptr), nbytes, max_slots,
                                                    path, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def pa_server_admit(h, desc):
    """Slot of the admitted run, or None when it does not fit now
    (PA_ERR_NOMEM) or no slot is free (PA_ERR_CAPACITY)."""
    arr, _keep = make_descs([desc])
    slot = C.c_int32(-1)
    st = lib().pa_server_admit(h, arr, C.byref(slot))
    if st in (PA_ERR_NOMEM, PA_ERR_CAPACITY):
        return None
    _chk("pa_server_admit", st, h, server=True)
    return slot.value


def pa_server_step(h, finished):
    n = C.c_int32(0)
    _chk("pa_server_step", lib().pa_server_step(h, _p(finished), C.byref(n)), h, server=True)
    return [int(x) for x in finished[:n.value]]


def pa_server_progress(h, slot):
    i = C.c_int32(0)
    _chk("pa_server_progress", lib().pa_server_progress(h, slot, C.byref(i)), h, server=True)
    return i.value


def pa_server_read_obs(h, slot, out, sync=True):
    _chk("pa_server_read_obs", lib().pa_server_read_obs(h, slot, C.c_void_p(out), int(sync)), h, server=True)


def pa_server_release(h, slot):
    _chk("pa_server_release", lib().pa_server_release(h, slot), h, server=True)


def pa_server_info(h):
    n, used, free = C.c_int32(0), C.c_size_t(0), C.c_size_t(0)
    _chk("pa_server_info", lib().pa_server_info(h, C.byref(n), C.byref(used), C.byref(free)), h, server=True)
    return dict(resident=n.value, bytes_used=used.value, largest_free=free.value)


def pa_server_destroy(h):
    _chk("pa_server_destroy", lib().pa_server_destroy(h))


# ------------------------------------------------------------ convenience

class Context:
    """A batch of PA runs on one GPU.  The device workspace is a torch uint8
    tensor owned by this object; the stream is torch's current stream (or
    the one given)."""

    def __init__(self, runs, repr_="msc", device="cuda", stream=None, static_workspace=False):
        """static_workspace=True creates the context with pa_create_static,
        in the library's own device array (no workspace tensor)."""
        import torch
        if isinstance(runs, dict):
            runs = [runs]
        self.runs = [dict(r) for r in runs]
        self.repr = REPRS[repr_]
        self.n_runs = len(runs)
        self.npop = 2 if any(r["overlap"] == PA_Q_TWO_POP for r in runs) else 1
        self.Kmax = max(len(r["beta"]) for r in runs)
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(dev):
                self.h = pa_create_static(self.runs, self.repr, self.stream.cuda_stream)
        else:
            nbytes = pa_workspace_size(self.runs, self.repr)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            ptr = (self.workspace.data_ptr() + 255) & ~255
            self.h = pa_create(self.runs, self.repr, ptr, nbytes, self.stream.cuda_stream)
        self.i = 0

    def close(self):
        if getattr(self, "h", None):
            pa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def anneal_step(self, i):
        pa_anneal_step(self.h, i)
        self.i = i

    def resample(self, i):
        pa_resample(self.h, i)

    def sweep(self, i):
        pa_sweep(self.h, i)

    def measure(self, i, read=False):
        out = np.zeros((self.n_runs, self.npop), PA_OBS_DTYPE) if read else None
        pa_measure(self.h, i, out)
        return out

    def step(self, i, read=False):
        self.anneal_step(i)
        self.resample(i)
        self.sweep(i)
        return self.measure(i, read)

    def run(self, i_begin, i_end):
        pa_run(self.h, i_begin, i_end)
        self.i = i_end - 1

    def obs(self):
        out = np.zeros((self.n_runs, self.npop, self.Kmax), PA_OBS_DTYPE)
        pa_read_obs(self.h, out)
        return out

    def weighted_average(self, M, kind=PA_W_FULL, pop=0):
        K = len(self.runs[0]["beta"])
        out = np.zeros((self.n_runs // M, K), PA_WAVG_DTYPE)
        pa_weighted_average(self.h, M, kind, pop, out)
        return out

    def weighted_qhist(self, M, kind=PA_W_FULL, pop=0):
        """Eq. (W_conf_q) per group of M runs: [n_runs/M, K, N+1]."""
        K = len(self.runs[0]["beta"])
        N = self.runs[0]["L"] ** 2
        out = np.zeros((self.n_runs // M, K, N + 1), np.float64)
        pa_weighted_qhist(self.h, M, kind, pop, out)
        return out

    def family_stats(self, pop=0):
        """rho_t, largest family and exclusion flags: [n_runs, K]."""
        out = np.zeros((self.n_runs, self.Kmax), PA_FAMSTAT_DTYPE)
        pa_family_stats(self.h, pop, out)
        return out

    def state(self, run=0, pop=0):
        d = self.runs[run]
        N = d["L"] ** 2
        s = np.zeros((d["R_cap"], N), np.int8)
        E = np.zeros(d["R_cap"], np.int32)
        f = np.zeros(d["R_cap"], np.int32)
        r = np.zeros(d["R_cap"], np.int32)
        Ri, Rp = pa_read_state(self.h, run, pop, s, E, f, r)
        return s[:Ri], E[:Ri], f[:Ri], r[:Rp]

    def pairing(self, run=0):
        """(status, pairs) of a permutation-pairing run at the last measured
        temperature: pairs[k] is the partner of replica k; status 1 when a
        family held more than R_i / 2 replicas (no pairing)."""
        out = np.zeros(self.runs[run]["R_cap"], np.int32)
        st, Ri = pa_read_pairing(self.h, run, out)
        return st, out[:Ri]

    def qhist(self, run=0):
        d = self.runs[run]
        npop = 2 if d["overlap"] == PA_Q_TWO_POP else 1
        out = np.zeros((npop, len(d["beta"]), d["L"] ** 2 + 1), np.int32)
        pa_read_qhist(self.h, run, out)
        return out

    def set_tuning(self, L, threads, groups_per_wg, dense_calls=3):
        pa_set_tuning(self.h, L, threads, groups_per_wg, dense_calls)

    def set_persistent(self, on):
        pa_set_persistent(self.h, on)

    def set_pooled(self, on):
        pa_set_pooled(self.h, on)

    def set_sweep_chunks(self, chunks):
        """Chunks of sweeps per item on the persistent grid (0: chosen per plan)."""
        pa_set_sweep_chunks(self.h, chunks)

    def sweep_chunks(self):
        """Chunks per item of the current sweep plan (1: whole items)."""
        return pa_get_sweep_chunks(self.h)

    def sweep_launches(self):
        """Launches of the batched sweep per temperature step."""
        return pa_get_sweep_launches(self.h)

    def tuning(self, L):
        return pa_get_tuning(self.h, L)

    def autotune(self, steps=3, cache_path=None):
        """Search launch shapes on this context's own next steps (its state
        is left unchanged); returns {'tried': n, 'rejected': n}."""
        return pa_autotune(self.h, steps, cache_path)

    def stats(self):
        """(word-site updates, Philox calls, attempted flips) of the sweeps."""
        w, c, f = (int(x) for x in pa_read_stats(self.h))
        return dict(words=w, calls=c, flips=f)

    def checkpoint(self):
        n = pa_checkpoint(self.h)
        buf = np.zeros(n, np.uint8)
        pa_checkpoint(self.h, buf)
        return buf

    def restore(self, buf):
        pa_restore(self.h, np.ascontiguousarray(buf, dtype=np.uint8))
