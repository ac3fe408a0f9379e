"""Oracle pins: Philox4x32-10, the Metropolis draw, threshold and reweighting
tables (CPU only)."""
import ctypes as C
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers or g++ not available")
    out = tmp_path_factory.mktemp("rr") / "rr.so"
    subprocess.run(["g++", "-O1", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", os.path.join(HERE, "rocrand_philox_ref.cpp"),
                    "-o", str(out)], check=True)
    lib = C.CDLL(str(out))

    def f(ctr, key):
        ctr = np.ascontiguousarray(ctr, np.uint32)
        key = np.ascontiguousarray(key, np.uint32)
        o = np.zeros((len(ctr), 4), np.uint32)
        lib.rr_philox(ctr.ctypes.data_as(C.c_void_p), key.ctypes.data_as(C.c_void_p),
                      o.ctypes.data_as(C.c_void_p), len(ctr))
        return o
    return f


def test_philox_matches_rocrand(rocrand_philox):
    """The oracle's Philox4x32-10 equals rocRAND's independent implementation
    of the same published generator on random and extreme (counter, key)."""
    rng = np.random.default_rng(2207_05535)
    n = 3000
    ctr = rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    ref = rocrand_philox(ctr, key)
    mine = np.array([oracle.philox4x32_10(ctr[i], key[i]) for i in range(n)])
    assert np.array_equal(mine, ref)


def test_sweep_draw_is_bit_plane_assembly():
    """u_j of replica j = 64g+b: bit 31-p is bit b of plane p; plane 2c is
    o0|o1<<32, plane 2c+1 is o2|o3<<32 of call c with counter
    (n | c<<20, g, i, 1<<28 | pop<<24 | s)."""
    seed = 0x1234_5678_9ABC
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (n, j, i, pop, s) in [(0, 0, 1, 0, 0), (77, 130, 5, 1, 9), (4095, 63, 199, 0, 3)]:
        g, b = divmod(j, 64)
        planes = []
        for c in range(16):
            o = oracle.philox4x32_10([n | (c << 20), g, i, (1 << 28) | (pop << 24) | s], key)
            planes.append(int(o[0]) | (int(o[1]) << 32))
            planes.append(int(o[2]) | (int(o[3]) << 32))
        u = 0
        for p in range(32):
            u |= ((planes[p] >> b) & 1) << (31 - p)
        assert oracle.sweep_draw(seed, n, j, i, pop, s) == u


def test_sweep_draw_uniform():
    """The assembled draws are uniform on [0, 2^32): chi-square of the top
    4 bits and the mean, over distinct (site, replica) counters."""
    seed = 0xABCDEF
    u = np.array([oracle.sweep_draw(seed, n, j, 3, 0, 1) for n in range(40) for j in range(128)],
                 dtype=np.float64)
    top = (u.astype(np.uint64) >> 28).astype(np.int64)
    cnt = np.bincount(top, minlength=16)
    exp_ = len(u) / 16
    chi2 = ((cnt - exp_) ** 2 / exp_).sum()
    assert chi2 < 45.0            # 15 dof, p ~ 1e-4
    z = (u.mean() / 2 ** 32 - 0.5) / math.sqrt(1 / 12 / len(u))
    assert abs(z) < 4.5


@pytest.mark.parametrize("beta", [0.0, 1e-9, 0.05, 0.4406868, 1.0, 3.0, 7.5, 40.0])
def test_sweep_threshold(beta):
    """T(beta, dE) / 2^32 is within 2^-32 below exp(-beta dE) (Metropolis
    acceptance, Sec. V A 1), with T = 2^32 exactly at beta = 0."""
    for dE in (4, 8):
        T = oracle.sweep_threshold(beta, dE)
        p = math.exp(-beta * dE)
        assert 0 <= T <= 2 ** 32
        assert 0.0 <= p - T / 2 ** 32 < 2.0 ** -32 + 1e-18
    if beta == 0.0:
        assert oracle.sweep_threshold(beta, 4) == 2 ** 32


def test_reweight_tables():
    """x_k = exp(-dbeta 4k) and X_k = floor(x_k 2^40): X_0 = 2^40, X monotone
    non-increasing, X_k / 2^40 within 2^-40 of x_k (Eq. (tauBoltz))."""
    for db in (0.0, 0.003, 0.005, 0.03, 0.5):
        prev = None
        for k in range(0, 300):
            x = oracle.reweight_x(db, k)
            X = oracle.reweight_X(db, k)
            assert x == pytest.approx(math.exp(-db * 4 * k), rel=1e-15, abs=0.0)
            assert 0 <= x * 2 ** 40 - X < 1.0
            if k == 0:
                assert X == 2 ** 40
            if prev is not None:
                assert X <= prev
            prev = X
