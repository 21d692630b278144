"""C-ABI checks that need no GPU: the library loads and exports every symbol
of include/rtrom.h, host-side quadrature, and argument validation (which
runs before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_19647_amd import rtrom
from paper_2603_19647_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "rtrom.h")).read()
    declared = set(re.findall(r"^(?:rtrom_status|void|const char\s*\*)\s*\*?\s*(rtrom_[a-z_]+)\s*\(",
                              hdr, re.M))
    assert declared == set(rtrom.EXPORTS), declared ^ set(rtrom.EXPORTS)
    L = rtrom.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n", [2, 4, 16, 64, 128])
def test_library_gauss_legendre(n):
    mu, w = rtrom.gauss_legendre(n)
    x, wn = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(mu, x, atol=1e-14)
    np.testing.assert_allclose(w, wn / 2, rtol=1e-10)
    np.testing.assert_array_equal(mu, -mu[::-1])
    np.testing.assert_array_equal(w, w[::-1])
    assert abs(w.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("nphi,nz", [(4, 2), (8, 4), (16, 8)])
def test_library_cl_quadrature_moments(nphi, nz):
    ox, oy, oz, w = rtrom.cl_quadrature(nphi, nz)
    assert abs(w.sum() - 1) < 1e-14
    for o in (ox, oy, oz):
        assert abs((w * o).sum()) < 1e-14
        assert abs((w * o * o).sum() - 1 / 3) < 1e-14


def _create_status(spec):
    keep = []
    d = rtrom.make_desc(spec, keep)
    h = ctypes.c_void_p()
    st = rtrom.lib().rtrom_create_problem(ctypes.byref(d), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [
    dict(dt=0.0), dict(dt=-1.0), dict(tol=0.0), dict(max_iter=0), dict(n_polar=3),
    dict(n_polar=0), dict(r_max=0), dict(r_max=21), dict(nx=0), dict(nx=5000),
    dict(eps_up=-1.0), dict(lx=0.0),
])
def test_invalid_descriptions_rejected_on_host(bad):
    spec = W.random_slab(1, 16, 4).replace(**bad)
    if "nx" in bad and bad["nx"] > 0:
        n = bad["nx"]
        spec = spec.replace(sigma_s=np.ones(n), sigma_a=np.ones(n), source=np.zeros(n))
    st, h = _create_status(spec)
    assert st == rtrom.EINVAL
    assert not h.value
    assert rtrom.last_error()


@pytest.mark.parametrize("field,value", [("sigma_s", np.nan), ("sigma_s", -1.0),
                                         ("sigma_a", np.inf), ("source", np.nan)])
def test_non_finite_or_negative_materials_rejected(field, value):
    spec = W.random_slab(2, 16, 4)
    arr = getattr(spec, field).copy()
    arr[3] = value
    st, _ = _create_status(spec.replace(**{field: arr}))
    assert st == rtrom.EINVAL


def test_2d_quadrature_order_checks():
    spec = W.random_plane(1, 4, 6, 2)  # N_phi not a multiple of 4
    st, _ = _create_status(spec)
    assert st == rtrom.EINVAL


def test_destroy_null_is_noop_and_null_args():
    rtrom.lib().rtrom_destroy_problem(None)
    out = np.zeros(4)
    assert rtrom.lib().rtrom_get_scalar_flux(None, out.ctypes.data_as(rtrom._D), 4) == rtrom.EINVAL
    assert rtrom.lib().rtrom_march(None, 1) == rtrom.EINVAL
    assert rtrom.lib().rtrom_march_batch(None, 0, 1) == rtrom.EINVAL


def test_estimate_bytes_scales_with_f():
    a = rtrom.estimate_bytes(W.random_slab(1, 1024, 16))
    b = rtrom.estimate_bytes(W.random_slab(1, 1024, 64))
    assert b - a >= 48 * 1024 * 8
    assert a > 16 * 1024 * 8


# ---- serving API: argument checks and failure paths (no device needed) ----

def _small_plane_spec():
    from paper_2603_19647_amd import workloads as W
    return W.random_plane(1, 16, 8, 4, nsteps=3)


def test_server_create_rejects_bad_arguments():
    with pytest.raises(rtrom.RtromError):
        rtrom.Server(hbm_budget_bytes=0)
    with pytest.raises(rtrom.RtromError):
        rtrom.Server(hbm_budget_bytes=1 << 30, max_slots=0)


@pytest.mark.gpu
def test_server_submit_validates_and_budget():
    s = rtrom.Server(hbm_budget_bytes=1 << 20, max_slots=1)
    try:
        spec = _small_plane_spec()
        with pytest.raises(rtrom.RtromError) as e:
            s.submit(spec.replace(dt=-1.0))
        assert e.value.status == rtrom.EINVAL
        big = spec.replace(nsteps=3)
        need = rtrom.estimate_bytes(big)
        assert need > (1 << 20)  # this small budget cannot hold the problem
        with pytest.raises(rtrom.RtromError) as e:
            s.submit(big)
        assert e.value.status == rtrom.ENOMEM
        with pytest.raises(rtrom.RtromError) as e:
            s.poll(12345)
        assert e.value.status == rtrom.EINVAL
    finally:
        s.close()


def test_variant_limits_rejected_on_the_host():
    """McClarren-Haut, BDF2 and sequential correction ROMs run on slabs of
    at most 2048 cells and on X-Y grids, DG-P1 on slabs of at most 1024 cells;
    unknown values are rejected.  All before any device call."""
    from paper_2603_19647_amd import rtrom
    from paper_2603_19647_amd import workloads as W
    bad = [W.random_slab(1, 2100, 8, precond="mh"), W.random_slab(1, 2100, 8, time_scheme="bdf2"),
           W.random_slab(1, 2100, 8, pc_levels=2),
           W.random_slab(1, 64, 8, pc_levels=5),
           W.random_slab(1, 64, 8, mh_rank=21),
           # DG-P1: slabs of at most 1024 cells, with DSA and backward Euler
           W.random_slab(1, 1025, 8, scheme="dg1"), W.random_plane(1, 8, 4, 2, scheme="dg1")]
    for s in bad:
        with pytest.raises(rtrom.RtromError) as e:
            rtrom.Problem(s)
        assert e.value.status == rtrom.EINVAL, s.name


def _run_logged(code, level):
    import subprocess
    import sys
    env = dict(os.environ)
    if level is None:
        env.pop("RTROM_LOG", None)
    else:
        env["RTROM_LOG"] = str(level)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=120)


def test_log_level_reports_errors_on_stderr():
    """RTROM_LOG=1 prints every error the library records (here a rejected
    description, before any device call) to stderr; unset, it prints nothing."""
    code = ("from paper_2603_19647_amd import rtrom, workloads as W\n"
            "try:\n"
            "    rtrom.Problem(W.random_slab(1, 64, 8, pc_levels=5))\n"
            "except rtrom.RtromError as e:\n"
            "    print('status', e.status)\n")
    r = _run_logged(code, 1)
    assert r.returncode == 0, r.stderr
    assert "status" in r.stdout
    assert "rtrom: error: pc_levels must be in 0..4" in r.stderr
    r = _run_logged(code, None)
    assert r.returncode == 0 and "rtrom:" not in r.stderr
