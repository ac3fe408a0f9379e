"""C ABI checks that need no GPU: libpa.so loads, exports every entry point
that include/pa.h declares, its record layouts match the binding, and
argument validation rejects bad descriptors before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2207_05535_amd as pa
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "pa_create" in names and "pa_weighted_average" in names and len(names) >= 15
    lib = C.CDLL(pa.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_record_layouts():
    assert pa.PA_OBS_DTYPE.itemsize == 136
    assert pa.PA_WAVG_DTYPE.itemsize == 120
    assert C.sizeof(pa.pa_run_desc) == 64
    assert pa.pa_run_desc.beta.offset == 40


def test_status_strings():
    for st in range(7):
        assert pa.status_str(st)


def _size(runs, repr_="int8"):
    arr, keep = pa.make_descs(runs)
    n = C.c_size_t(0)
    return pa.lib().pa_workspace_size(arr, len(runs), pa.REPRS[repr_], C.byref(n)), n.value


def test_workspace_size_valid_and_monotone():
    d = W.fm_L8_R1000()
    st, n8 = _size([d], "int8")
    assert st == 0 and n8 > 2 * 1000 * 64
    st, nm = _size([d], "msc")
    assert st == 0 and 0 < nm < n8
    st, n2 = _size([d, d], "msc")
    assert st == 0 and n2 > nm


@pytest.mark.parametrize("bad", [
    dict(L=7), dict(L=2), dict(L=2048), dict(theta=-2), dict(R=0), dict(R_cap=10),
    dict(theta=-1, model=1), dict(theta=-1, L=32), dict(theta=-1, overlap=1),   # theta = infinity: FM, L <= 30, no q
    dict(R_cap=2000),                      # multinomial needs R_cap == R
    dict(model=3), dict(resampling=5), dict(overlap=7), dict(qhist=2),
    dict(beta=[0.1, 0.2, 0.3]),            # beta_0 must be 0
    dict(beta=[0.0]),                      # K >= 2
    dict(beta=[0.0, float("nan")]),
    dict(beta=[0.0, 0.3, 0.2, 0.4]),       # a schedule that heats is rejected
    dict(R=1 << 23, R_cap=1 << 23),
])
def test_workspace_size_rejects(bad):
    d = W.with_(W.fm_L8_R1000(), **bad)
    st, _ = _size([d])
    assert st == pa.PA_ERR_ARG


def test_calibration_validates_before_the_device():
    lib = pa.lib()
    out = C.c_double(0.0)
    assert lib.pa_calibrate_philox(None, 0, C.byref(out)) == pa.PA_ERR_ARG
    assert lib.pa_calibrate_philox(None, (1 << 20) + 1, C.byref(out)) == pa.PA_ERR_ARG
    assert lib.pa_calibrate_philox(None, 16, None) == pa.PA_ERR_ARG


def test_exact_dos_validates_before_computing():
    lib = pa.lib()
    buf = np.zeros(2 * 145, np.uint64)
    for L in (2, 3, 12):
        assert lib.pa_exact_dos(L, buf.ctypes.data) == pa.PA_ERR_ARG
    assert lib.pa_exact_dos(8, None) == pa.PA_ERR_ARG
    wide = np.zeros(16 * 1025, np.uint64)
    for L, limbs in ((32, 17), (7, 2), (16, 4), (16, 0)):     # L even <= 30; limbs >= N/64 + 1
        assert lib.pa_exact_dos_wide(L, limbs, wide.ctypes.data) == pa.PA_ERR_ARG
    assert lib.pa_exact_dos_wide(16, 5, None) == pa.PA_ERR_ARG


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 16])
def test_library_dos_equals_oracle(L):
    """The library's density of states (modular product formula, host code)
    equals the oracle's (transfer matrix for L <= 8, high-precision product
    formula beyond) exactly."""
    from oracle import dos
    import oracle
    ref = oracle.exact_dos(L) if L <= 8 else list(dos.fm_dos(L))
    assert pa.pa_exact_dos(L) == ref


def test_msc_lattice_limit():
    d = W.run_desc(256, W.FM, R=64, K=3, beta_f=0.1)
    assert _size([d], "int8")[0] == 0
    assert _size([d], "msc")[0] == pa.PA_ERR_ARG


def test_create_validates_before_device():
    d = W.fm_L8_R1000()
    arr, keep = pa.make_descs([d])
    h = C.c_void_p()
    L = pa.lib()
    # null workspace / misaligned / too small: rejected without touching a device
    assert L.pa_create(arr, 1, 0, None, 1 << 30, None, C.byref(h)) == pa.PA_ERR_ARG
    assert L.pa_create(arr, 1, 0, C.c_void_p(0x1001), 1 << 30, None, C.byref(h)) == pa.PA_ERR_ARG
    assert L.pa_create(arr, 1, 0, C.c_void_p(0x10000), 16, None, C.byref(h)) == pa.PA_ERR_NOMEM
    assert L.pa_create(arr, 0, 0, C.c_void_p(0x10000), 1 << 30, None, C.byref(h)) == pa.PA_ERR_ARG
    assert L.pa_create(arr, 1, 9, C.c_void_p(0x10000), 1 << 30, None, C.byref(h)) == pa.PA_ERR_ARG
    for f in ("pa_anneal_step", "pa_resample", "pa_sweep"):
        assert getattr(L, f)(None, 1) == pa.PA_ERR_ARG
    assert L.pa_measure(None, 1, None) == pa.PA_ERR_ARG
    assert L.pa_run(None, 1, 2) == pa.PA_ERR_ARG
    assert L.pa_destroy(None) == pa.PA_ERR_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pa, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pa, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pa.lib()


def test_server_footprint_and_validation():
    d = W.run_desc(16, W.EA_PMJ, R=5000, K=21, overlap=W.Q_INDEX_SHIFT)
    fm = pa.pa_server_footprint(d, "msc")
    f8 = pa.pa_server_footprint(d, "int8")
    assert 0 < fm < f8
    # the block grows with R and with a second population
    assert pa.pa_server_footprint(W.with_(d, R=10000, R_cap=10000), "msc") > fm
    assert pa.pa_server_footprint(W.with_(d, overlap=W.Q_TWO_POP), "msc") > fm
    with pytest.raises(pa.PAError):
        pa.pa_server_footprint(W.with_(d, L=7), "msc")
    lib = pa.lib()
    h = C.c_void_p()
    # rejected before any device call: no arena, misaligned arena, no slots
    assert lib.pa_server_create(pa.PA_MSC64, None, 1 << 20, 4, None, None, C.byref(h)) == pa.PA_ERR_ARG
    assert lib.pa_server_create(pa.PA_MSC64, C.c_void_p(4096 + 8), 1 << 20, 4, None, None,
                                C.byref(h)) == pa.PA_ERR_ARG
    assert lib.pa_server_create(pa.PA_MSC64, C.c_void_p(4096), 1 << 20, 0, None, None,
                                C.byref(h)) == pa.PA_ERR_ARG
    assert lib.pa_server_create(pa.PA_MSC64, C.c_void_p(4096), 1024, 4, None, None,
                                C.byref(h)) == pa.PA_ERR_NOMEM
    assert lib.pa_server_step(None, None, None) == pa.PA_ERR_ARG
    assert lib.pa_server_release(None, 0) == pa.PA_ERR_ARG


def test_tuning_calls_validate_before_device():
    lib = pa.lib()
    assert lib.pa_autotune(None, 3, None, None, None) == pa.PA_ERR_ARG
    assert lib.pa_set_persistent(None, 1) == pa.PA_ERR_ARG
    assert lib.pa_get_tuning(None, 16, None, None, None, None, None) == pa.PA_ERR_ARG
    assert lib.pa_set_pooled(None, 1) == pa.PA_ERR_ARG
