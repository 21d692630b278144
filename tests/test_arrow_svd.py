"""CPU tests of the secular core SVD (rt_arrow.h), built for the host from the
same header the device uses, against numpy's SVD of the incremental-SVD core
K = [[diag S, a], [0, nu]] and its rank-deficient form [diag S, a]."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2603_19647_amd", "csrc")


@pytest.fixture(scope="module")
def arrow():
    d = tempfile.mkdtemp(prefix="arrow_")
    so = os.path.join(d, "arrow_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                           os.path.join(HERE, "arrow_host.cpp"), "-o", so])
    lib = ctypes.CDLL(so)
    P = ctypes.POINTER(ctypes.c_double)
    lib.arrow_host.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_double, P, P, P]
    lib.arrow_host.restype = ctypes.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def run(lib, S, a, nu, deficient=False):
    r = len(S)
    rows = r if deficient else r + 1
    sv = np.zeros(rows)
    U = np.zeros((rows, rows))
    V = np.zeros((r + 1, rows))
    ok = lib.arrow_host(r, rows, _p(np.ascontiguousarray(S)), _p(np.ascontiguousarray(a)), nu, _p(sv), _p(U), _p(V))
    return ok, sv, U, V


def core(S, a, nu, deficient=False):
    r = len(S)
    K = np.zeros((r if deficient else r + 1, r + 1))
    K[:r, :r] = np.diag(S)
    K[:r, r] = a
    if not deficient:
        K[r, r] = nu
    return K


def check(lib, S, a, nu, deficient=False, tol=2e-13):
    ok, sv, U, V = run(lib, S, a, nu, deficient)
    assert ok
    K = core(S, a, nu, deficient)
    ref = np.linalg.svd(K, compute_uv=False)
    nK = ref[0]
    # singular values: absolute to ||K|| eps, relative for the well-separated large ones
    assert np.max(np.abs(sv - ref)) <= tol * nK, (sv, ref)
    n = U.shape[1]
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= tol * 10
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= tol * 10
    assert np.max(np.abs(K @ V - U * sv)) <= tol * nK
    return sv


@pytest.mark.parametrize("seed", range(40))
def test_random_cores(arrow, seed):
    rng = np.random.default_rng(seed)
    r = int(rng.integers(1, 21))
    decay = rng.choice([0.9, 0.5, 0.3, 0.1])
    S = np.sort(decay ** np.arange(r) * rng.uniform(0.5, 2.0, r))[::-1].copy()
    a = rng.standard_normal(r) * 10.0 ** rng.uniform(-8, 0, r)
    nu = 10.0 ** rng.uniform(-10, 0)
    check(arrow, S, a, nu)
    check(arrow, S, a, nu, deficient=True)


def test_deflated_couplings(arrow):
    S = 0.5 ** np.arange(12)
    a = np.full(12, 1e-3)
    a[[2, 7]] = 1e-30   # below rounding: deflated rows
    a[5] = 1e-12        # small but resolved
    check(arrow, S, a, 1e-2)
    check(arrow, S, a, 0.0, deficient=True)


def test_rank_one_and_small_nu(arrow):
    check(arrow, np.array([3.0]), np.array([0.7]), 1e-9)
    check(arrow, np.array([3.0]), np.array([0.7]), 0.0, deficient=True)
    S = np.array([1.0, 1e-3, 1e-6])
    check(arrow, S, np.array([1e-2, 1e-4, 1e-9]), 1e-11)


def test_coinciding_singular_values_decline(arrow):
    S = np.array([1.0, 0.5, 0.5, 0.1])
    ok, *_ = run(arrow, S, np.array([0.1, 0.2, 0.3, 0.4]), 0.05)
    assert ok == 0
