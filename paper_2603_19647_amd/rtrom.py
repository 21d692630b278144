"""Python binding of librtrom.so (ctypes; argument marshalling only).

Every step of the method runs in the HIP library.  This module only converts
``ProblemSpec`` objects into ``rtrom_problem_desc`` structs and numpy buffers,
and raises when the library is missing or reports an error: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtrom.so")

OK, EINVAL, ENOMEM, ENOCONV, EDEVICE, EBUSY = 0, -1, -2, -3, -4, -5
METHOD = {"si_dsa": 0, "rom": 1, "si": 2}
PRECISION = {"fp64": 0, "mixed": 1}
PRECOND = {"dsa": 0, "mh": 1}
TIME_SCHEME = {"be": 0, "bdf2": 1}
SCHEME = {"fv": 0, "dg1": 1}
F_ABS_UP_NORM = 0x1
F_SINGLE_WG = 0x2

_D = ctypes.POINTER(ctypes.c_double)


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("n_polar", ctypes.c_int32), ("n_azim", ctypes.c_int32),
        ("sigma_s", _D), ("sigma_a", _D), ("source", _D), ("f0", _D),
        ("inflow", ctypes.c_double * 4),
        ("dt", ctypes.c_double), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eps_ig", ctypes.c_double), ("eps_pc", ctypes.c_double), ("eps_up", ctypes.c_double),
        ("r_max", ctypes.c_int32), ("flags", ctypes.c_uint64),
        ("precond", ctypes.c_int32), ("time_scheme", ctypes.c_int32),
        ("pc_levels", ctypes.c_int32), ("mh_rank", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("pad_", ctypes.c_int32), ("lu_tol", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("si_iters_total", ctypes.c_int64), ("sweeps_total", ctypes.c_int64),
        ("si_iters_last", ctypes.c_int32), ("phase", ctypes.c_int32),
        ("n0", ctypes.c_int32), ("n1", ctypes.c_int32),
        ("rank_ig", ctypes.c_int32), ("rank_pc", ctypes.c_int32),
        ("nonconverged_steps", ctypes.c_int32), ("rom_fallbacks", ctypes.c_int32),
        ("ig_updates", ctypes.c_int64), ("pc_updates", ctypes.c_int64), ("fp32_sweeps", ctypes.c_int64),
        ("last_residual", ctypes.c_double), ("t_total_s", ctypes.c_double),
        ("dsa_iters", ctypes.c_int32), ("reserved_", ctypes.c_int32),
    ]


class StepRecord(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("phase", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("ig_update", ctypes.c_int32), ("pc_update", ctypes.c_int32),
        ("rank_ig", ctypes.c_int32), ("rank_pc", ctypes.c_int32), ("fallback", ctypes.c_int32),
        ("e_ig", ctypes.c_double), ("e_pc", ctypes.c_double), ("residual", ctypes.c_double),
    ]


class ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("steps_per_tick", ctypes.c_int32)]


class RtromError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rtrom status {status}: {msg}")
        self.status = status


# every symbol declared in include/rtrom.h
EXPORTS = (
    "rtrom_create_problem", "rtrom_step", "rtrom_march", "rtrom_march_batch", "rtrom_march_batch_noalloc",
    "rtrom_get_scalar_flux", "rtrom_get_angular_flux", "rtrom_get_rhs", "rtrom_get_quadrature",
    "rtrom_gauss_legendre", "rtrom_cl_quadrature", "rtrom_stats_get", "rtrom_get_levels", "rtrom_get_history",
    "rtrom_set_inflow", "rtrom_set_stream", "rtrom_device_bytes", "rtrom_estimate_bytes",
    "rtrom_destroy_problem", "rtrom_last_error",
    "rtrom_server_create", "rtrom_server_submit", "rtrom_server_poll", "rtrom_server_drain",
    "rtrom_server_fetch", "rtrom_server_destroy", "rtrom_profile_enable", "rtrom_profile_read",
)
KERNEL_KINDS = ("slab_si", "slab_fpass", "post", "plane_sweep", "plane_dsa", "plane_fpass", "plane_other",
                "rom_update")

_lib = None


def lib():
    """Load librtrom.so; raise loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2603_19647_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.rtrom_last_error.restype = ctypes.c_char_p
    L.rtrom_create_problem.argtypes = [ctypes.POINTER(Desc), pp]
    L.rtrom_step.argtypes = [vp]
    L.rtrom_march.argtypes = [vp, i32]
    L.rtrom_march_batch.argtypes = [ctypes.POINTER(ctypes.c_void_p), i32, i32]
    L.rtrom_march_batch_noalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), i32, i32]
    L.rtrom_get_scalar_flux.argtypes = [vp, _D, i64]
    L.rtrom_get_angular_flux.argtypes = [vp, _D, i64]
    L.rtrom_get_rhs.argtypes = [vp, _D, i64]
    L.rtrom_get_quadrature.argtypes = [vp, _D, _D, _D, _D, i64]
    L.rtrom_gauss_legendre.argtypes = [i32, _D, _D]
    L.rtrom_cl_quadrature.argtypes = [i32, i32, _D, _D, _D, _D]
    L.rtrom_stats_get.argtypes = [vp, ctypes.POINTER(Stats)]
    L.rtrom_get_history.argtypes = [vp, ctypes.POINTER(StepRecord), i64, ctypes.POINTER(i64)]
    L.rtrom_get_levels.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32, ctypes.POINTER(i32)]
    L.rtrom_set_inflow.argtypes = [vp, _D]
    L.rtrom_set_stream.argtypes = [vp, vp]
    L.rtrom_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.rtrom_estimate_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_uint64)]
    L.rtrom_destroy_problem.argtypes = [vp]
    L.rtrom_destroy_problem.restype = None
    L.rtrom_server_create.argtypes = [ctypes.POINTER(ServerDesc), pp]
    L.rtrom_server_submit.argtypes = [vp, ctypes.POINTER(Desc), i32, ctypes.POINTER(ctypes.c_uint64)]
    L.rtrom_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32)]
    L.rtrom_server_drain.argtypes = [vp]
    L.rtrom_server_fetch.argtypes = [vp, ctypes.c_uint64, _D, i64, ctypes.POINTER(Stats), _D, i64, _D]
    L.rtrom_server_destroy.argtypes = [vp]
    L.rtrom_server_destroy.restype = None
    L.rtrom_profile_enable.argtypes = [i32]
    L.rtrom_profile_read.argtypes = [_D, ctypes.POINTER(i64), i32]
    _lib = L
    return L


def last_error() -> str:
    return lib().rtrom_last_error().decode(errors="replace")


def _check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise RtromError(status, last_error())
    return status


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def make_desc(spec, keep: list) -> Desc:
    """Fill an rtrom_problem_desc from a ProblemSpec; `keep` holds the arrays."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (spec.sigma_s, spec.sigma_a, spec.source)]
    keep.extend(arrs)
    d = Desc()
    d.dim, d.nx, d.ny = spec.dim, spec.nx, spec.ny
    d.lx, d.ly = spec.lx, spec.ly
    d.n_polar, d.n_azim = spec.n_polar, spec.n_azim
    d.sigma_s, d.sigma_a, d.source = (_p(a) for a in arrs)
    if spec.f0 is not None:
        f0 = np.ascontiguousarray(spec.f0, dtype=np.float64)
        keep.append(f0)
        d.f0 = _p(f0)
    else:
        d.f0 = _D()
    for k in range(4):
        d.inflow[k] = float(spec.inflow[k])
    d.dt, d.tol, d.max_iter = spec.dt, spec.tol, spec.max_iter
    d.method = METHOD[spec.method]
    d.precision = PRECISION[spec.precision]
    d.eps_ig, d.eps_pc, d.eps_up = spec.eps_ig, spec.eps_pc, spec.eps_up
    d.r_max = spec.r_max
    d.flags = (F_ABS_UP_NORM if spec.abs_up_norm else 0) | (F_SINGLE_WG if spec.single_wg else 0)
    d.precond = PRECOND[spec.precond]
    d.time_scheme = TIME_SCHEME[spec.time_scheme]
    d.pc_levels = int(spec.pc_levels)
    d.mh_rank = int(spec.mh_rank)
    d.scheme = SCHEME[spec.scheme]
    d.lu_tol = float(spec.lu_tol)
    return d


def gauss_legendre(n: int):
    mu, w = np.zeros(n), np.zeros(n)
    _check(lib().rtrom_gauss_legendre(n, _p(mu), _p(w)))
    return mu, w


def cl_quadrature(nphi: int, nz: int):
    nv = nphi * nz
    ox, oy, oz, w = (np.zeros(nv) for _ in range(4))
    _check(lib().rtrom_cl_quadrature(nphi, nz, _p(ox), _p(oy), _p(oz), _p(w)))
    return ox, oy, oz, w


def estimate_bytes(spec) -> int:
    keep: list = []
    d = make_desc(spec, keep)
    out = ctypes.c_uint64()
    _check(lib().rtrom_estimate_bytes(ctypes.byref(d), ctypes.byref(out)))
    return int(out.value)


class Problem:
    """A time-marching problem resident on the GPU."""

    def __init__(self, spec, **overrides):
        if overrides:
            spec = spec.replace(**overrides)
        self.spec = spec
        keep: list = []
        d = make_desc(spec, keep)
        h = ctypes.c_void_p()
        _check(lib().rtrom_create_problem(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.nc = spec.nx * spec.ny * (2 if spec.scheme == "dg1" else 1)  # unknowns of rho
        self.nv = spec.nord

    # -- marching ----------------------------------------------------------
    def step(self) -> int:
        return _check(lib().rtrom_step(self.h), allow=(OK, ENOCONV))

    def march(self, nsteps: int) -> int:
        return _check(lib().rtrom_march(self.h, int(nsteps)), allow=(OK, ENOCONV))

    # -- state ---------------------------------------------------------------
    def rho(self) -> np.ndarray:
        out = np.zeros(self.nc)
        _check(lib().rtrom_get_scalar_flux(self.h, _p(out), out.size))
        return out

    def f(self) -> np.ndarray:
        out = np.zeros(self.nc * self.nv)
        _check(lib().rtrom_get_angular_flux(self.h, _p(out), out.size))
        return out.reshape(self.nv, self.nc)

    def rhs(self) -> np.ndarray:
        out = np.zeros(self.nc)
        _check(lib().rtrom_get_rhs(self.h, _p(out), out.size))
        return out

    def quadrature(self):
        ox, oy, oz, w = (np.zeros(self.nv) for _ in range(4))
        _check(lib().rtrom_get_quadrature(self.h, _p(ox), _p(oy), _p(oz), _p(w), self.nv))
        return ox, oy, oz, w

    def stats(self) -> dict:
        s = Stats()
        _check(lib().rtrom_stats_get(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def levels(self) -> List[dict]:
        """Per correction ROM level: complete flag, N_l, rank, updates."""
        a = (ctypes.c_int64 * 16)()
        nl = ctypes.c_int32()
        _check(lib().rtrom_get_levels(self.h, a, 16, ctypes.byref(nl)))
        return [dict(flag=int(a[4 * k]), n=int(a[4 * k + 1]), rank=int(a[4 * k + 2]), updates=int(a[4 * k + 3]))
                for k in range(nl.value)]

    def history(self, n: Optional[int] = None) -> dict:
        n = self.stats()["steps"] if n is None else n
        arr = (StepRecord * max(int(n), 1))()
        wr = ctypes.c_int64()
        _check(lib().rtrom_get_history(self.h, arr, int(n), ctypes.byref(wr)))
        m = wr.value
        return {k: np.array([getattr(arr[i], k) for i in range(m)]) for k, _ in StepRecord._fields_}

    def set_inflow(self, g: Sequence[float]):
        g = np.ascontiguousarray(g, dtype=np.float64)
        _check(lib().rtrom_set_inflow(self.h, _p(g)))

    def set_stream(self, stream=None):
        """Launch on a HIP stream: an int handle, a torch.cuda.Stream, or None."""
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        _check(lib().rtrom_set_stream(self.h, ctypes.c_void_p(stream) if stream else None))

    def device_bytes(self) -> int:
        out = ctypes.c_uint64()
        _check(lib().rtrom_device_bytes(self.h, ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if getattr(self, "h", None):
            lib().rtrom_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    _check(lib().rtrom_profile_enable(int(bool(on))))


def profile_read() -> dict:
    n = len(KERNEL_KINDS)
    sec = np.zeros(n)
    cnt = (ctypes.c_int64 * n)()
    _check(lib().rtrom_profile_read(_p(sec), cnt, n))
    return {k: (float(sec[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}


def march_batch(problems: Sequence[Problem], nsteps: int) -> int:
    arr = (ctypes.c_void_p * len(problems))(*[p.h.value for p in problems])
    return _check(lib().rtrom_march_batch(arr, len(problems), int(nsteps)), allow=(OK, ENOCONV))


def march_batch_noalloc(problems: Sequence[Problem], nsteps: int) -> int:
    """rtrom_march_batch_noalloc: the batch march without device allocation."""
    arr = (ctypes.c_void_p * len(problems))(*[p.h.value for p in problems])
    return _check(lib().rtrom_march_batch_noalloc(arr, len(problems), int(nsteps)), allow=(OK, ENOCONV))


class Server:
    """Continuous-batching server of independent problems (see rtrom.h)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, device: int = 0,
                 steps_per_tick: int = 1):
        d = ServerDesc(int(hbm_budget_bytes), int(max_slots), int(device), int(steps_per_tick))
        h = ctypes.c_void_p()
        _check(lib().rtrom_server_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self._specs = {}

    def submit(self, spec, nsteps: Optional[int] = None) -> int:
        keep: list = []
        d = make_desc(spec, keep)
        t = ctypes.c_uint64()
        n = spec.nsteps if nsteps is None else nsteps
        _check(lib().rtrom_server_submit(self.h, ctypes.byref(d), int(n), ctypes.byref(t)))
        self._specs[t.value] = (spec, n)
        return t.value

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int32()
        _check(lib().rtrom_server_poll(self.h, ticket, ctypes.byref(s)))
        return s.value

    def drain(self):
        _check(lib().rtrom_server_drain(self.h))

    def fetch(self, ticket: int):
        spec, n = self._specs[ticket]
        rho = np.zeros(spec.nx * spec.ny * (2 if spec.scheme == "dg1" else 1))  # unknowns
        lat = np.zeros(max(n, 1))
        mlat = ctypes.c_double()
        st = Stats()
        _check(lib().rtrom_server_fetch(self.h, ticket, _p(rho), rho.size, ctypes.byref(st), _p(lat),
                                        lat.size, ctypes.byref(mlat)), allow=(OK, ENOCONV))
        del self._specs[ticket]
        return rho, {k: getattr(st, k) for k, _ in Stats._fields_}, lat[:n], mlat.value

    def close(self):
        if getattr(self, "h", None):
            lib().rtrom_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
