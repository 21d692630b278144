"""ctypes handle on the FP64 CPU oracle (``rtrom_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the HIP library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtrom_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

METHOD = {"si_dsa": 0, "rom": 1, "si": 2}
PRECOND = {"dsa": 0, "mh": 1}
TIME_SCHEME = {"be": 0, "bdf2": 1}
SCHEME = {"fv": 0, "dg1": 1}
_D = ctypes.POINTER(ctypes.c_double)


class OrcDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("n_polar", ctypes.c_int32), ("n_azim", ctypes.c_int32),
        ("sigma_s", _D), ("sigma_a", _D), ("source", _D), ("f0", _D),
        ("inflow", ctypes.c_double * 4),
        ("dt", ctypes.c_double), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32),
        ("eps_ig", ctypes.c_double), ("eps_pc", ctypes.c_double), ("eps_up", ctypes.c_double),
        ("r_max", ctypes.c_int32), ("abs_up_norm", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("time_scheme", ctypes.c_int32),
        ("pc_levels", ctypes.c_int32), ("mh_rank", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("pad_", ctypes.c_int32), ("lu_tol", ctypes.c_double),
    ]


class StepRec(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("phase", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("ig_update", ctypes.c_int32), ("pc_update", ctypes.c_int32),
        ("rank_ig", ctypes.c_int32), ("rank_pc", ctypes.c_int32), ("fallback", ctypes.c_int32),
        ("e_ig", ctypes.c_double), ("e_pc", ctypes.c_double), ("residual", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    L.orc_create.restype = vp
    L.orc_create.argtypes = [ctypes.POINTER(OrcDesc)]
    L.orc_destroy.argtypes = [vp]
    L.orc_step.argtypes = [vp]
    L.orc_march.argtypes = [vp, ctypes.c_int]
    for nm in ("orc_get_rho", "orc_get_f", "orc_get_bt"):
        getattr(L, nm).argtypes = [vp, _D]
    L.orc_get_quadrature.argtypes = [vp, _D, _D, _D, _D]
    L.orc_get_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.orc_get_history.argtypes = [vp, ctypes.POINTER(StepRec), ctypes.c_int64]
    L.orc_ncells.argtypes = [vp]
    L.orc_nord.argtypes = [vp]
    L.orc_set_inflow.argtypes = [vp, _D]
    L.orc_apply_TSs.argtypes = [vp, _D, _D]
    L.orc_dsa_apply_inverse.argtypes = [vp, _D, _D]
    L.orc_dsa_entry.restype = ctypes.c_double
    L.orc_dsa_entry.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.orc_sweep.argtypes = [vp, ctypes.c_int, _D, ctypes.c_int, _D]
    L.orc_gauss_legendre.argtypes = [ctypes.c_int, _D, _D]
    L.orc_cl_quadrature.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
    L.orc_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
    L.orc_lu_factor.argtypes = [ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
    L.orc_lu_solve.argtypes = [ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int), _D]
    L.orc_get_step_vectors.argtypes = [vp, _D, _D, _D, _D]
    L.orc_get_rom.argtypes = [vp, ctypes.c_int, _D, _D, _D]
    L.orc_rom_new.restype = vp
    L.orc_rom_new.argtypes = [ctypes.c_int, ctypes.c_int]
    L.orc_rom_delete.argtypes = [vp]
    L.orc_rom_push.argtypes = [vp, _D, _D, ctypes.c_int, ctypes.c_double]
    L.orc_rom_rank.argtypes = [vp]
    L.orc_rom_lu_ok.argtypes = [vp]
    L.orc_rom_get.argtypes = [vp, _D, _D, _D]
    L.orc_rom_reduced.argtypes = [vp, _D]
    L.orc_rom_solve.argtypes = [vp, _D, _D]
    L.orc_mh_new.restype = vp
    L.orc_mh_new.argtypes = [ctypes.c_int, ctypes.c_int]
    L.orc_mh_delete.argtypes = [vp]
    L.orc_mh_push.argtypes = [vp, _D, _D]
    L.orc_mh_size.argtypes = [vp]
    L.orc_mh_correct.argtypes = [vp, _D, _D]
    L.orc_get_levels.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    assert L.orc_step_rec_size() == ctypes.sizeof(StepRec)
    assert L.orc_desc_size() == ctypes.sizeof(OrcDesc)
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def gauss_legendre(n: int):
    mu = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _p(mu), _p(w))
    return mu, w


def cl_quadrature(nphi: int, nz: int):
    nv = nphi * nz
    ox, oy, oz, w = (np.zeros(nv) for _ in range(4))
    lib().orc_cl_quadrature(nphi, nz, _p(ox), _p(oy), _p(oz), _p(w))
    return ox, oy, oz, w


def jacobi_svd(K: np.ndarray):
    K = np.ascontiguousarray(K, dtype=np.float64)
    rows, cols = K.shape
    Uc = np.zeros((rows, cols))
    s = np.zeros(cols)
    V = np.zeros((cols, cols))
    lib().orc_jacobi_svd(rows, cols, _p(K), _p(Uc), _p(s), _p(V))
    return Uc, s, V


def lu_solve(A: np.ndarray, b: np.ndarray):
    n = A.shape[0]
    LU = np.ascontiguousarray(A, dtype=np.float64).copy()
    piv = (ctypes.c_int * n)()
    bad = lib().orc_lu_factor(n, _p(LU), piv)
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    lib().orc_lu_solve(n, _p(LU), piv, _p(x))
    return x, bool(bad)


class Rom:
    """Standalone incremental-SVD / DMD object (App. B)."""

    def __init__(self, nc: int, rmax: int):
        self.nc = nc
        self.h = lib().orc_rom_new(nc, rmax)

    def push(self, x, b, truncate=False, eps=0.0) -> int:
        x = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        return lib().orc_rom_push(self.h, _p(x), _p(b), int(truncate), float(eps))

    @property
    def rank(self) -> int:
        return lib().orc_rom_rank(self.h)

    @property
    def lu_ok(self) -> bool:
        return bool(lib().orc_rom_lu_ok(self.h))

    def get(self):
        r = self.rank
        U = np.zeros((r, self.nc))
        W = np.zeros((r, self.nc))
        S = np.zeros(r)
        lib().orc_rom_get(self.h, _p(U), _p(S), _p(W))
        return U.T.copy(), S, W.T.copy()

    def reduced(self):
        r = self.rank
        A = np.zeros((r, r))
        lib().orc_rom_reduced(self.h, _p(A))
        return A

    def solve(self, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        out = np.zeros(self.nc)
        lib().orc_rom_solve(self.h, _p(rhs), _p(out))
        return out

    def __del__(self):
        try:
            lib().orc_rom_delete(self.h)
        except Exception:
            pass


class MhModel:
    """Standalone McClarren-Haut model (DMD of the sweep operator from
    iteration pairs, Sec. 3.3)."""

    def __init__(self, nc: int, cap: int):
        self.nc = nc
        self.h = lib().orc_mh_new(nc, cap)
        if not self.h:
            raise ValueError("bad McClarren-Haut model size")

    def push(self, x, z) -> bool:
        """Add (x, z = T Sigma_s x); False when the pair was skipped."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        return lib().orc_mh_push(self.h, _p(x), _p(z)) == 0

    @property
    def size(self) -> int:
        return lib().orc_mh_size(self.h)

    def correct(self, r):
        """(correction, applied) for the SI residual r."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(self.nc)
        bad = lib().orc_mh_correct(self.h, _p(r), _p(out))
        return out, bad == 0

    def __del__(self):
        try:
            lib().orc_mh_delete(self.h)
        except Exception:
            pass


class OracleProblem:
    """One oracle time-marching problem built from a ``ProblemSpec``."""

    def __init__(self, spec, method: Optional[str] = None):
        self.spec = spec
        m = spec.method if method is None else method
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (spec.sigma_s, spec.sigma_a, spec.source)]
        f0 = None if spec.f0 is None else np.ascontiguousarray(spec.f0, dtype=np.float64)
        self._keep.append(f0)
        d = OrcDesc()
        d.dim, d.nx, d.ny = spec.dim, spec.nx, spec.ny
        d.lx, d.ly = spec.lx, spec.ly
        d.n_polar, d.n_azim = spec.n_polar, spec.n_azim
        d.sigma_s, d.sigma_a, d.source = (_p(a) for a in self._keep[:3])
        d.f0 = _p(f0) if f0 is not None else _D()
        for k in range(4):
            d.inflow[k] = float(spec.inflow[k])
        d.dt, d.tol, d.max_iter = spec.dt, spec.tol, spec.max_iter
        d.method = METHOD[m]
        d.eps_ig, d.eps_pc, d.eps_up = spec.eps_ig, spec.eps_pc, spec.eps_up
        d.r_max = spec.r_max
        d.abs_up_norm = int(spec.abs_up_norm)
        d.precond = PRECOND[spec.precond]
        d.time_scheme = TIME_SCHEME[spec.time_scheme]
        d.pc_levels = int(spec.pc_levels)
        d.mh_rank = int(spec.mh_rank)
        d.scheme = SCHEME[spec.scheme]
        d.lu_tol = float(spec.lu_tol)
        self.h = lib().orc_create(ctypes.byref(d))
        if not self.h:
            raise ValueError("oracle rejected the problem description")
        self.nc = lib().orc_ncells(self.h)
        self.nv = lib().orc_nord(self.h)

    def step(self) -> int:
        return lib().orc_step(self.h)

    def march(self, n: int) -> int:
        return lib().orc_march(self.h, int(n))

    def rho(self):
        out = np.zeros(self.nc)
        lib().orc_get_rho(self.h, _p(out))
        return out

    def f(self):
        out = np.zeros(self.nc * self.nv)
        lib().orc_get_f(self.h, _p(out))
        return out.reshape(self.nv, self.nc)

    def bt(self):
        out = np.zeros(self.nc)
        lib().orc_get_bt(self.h, _p(out))
        return out

    def quadrature(self):
        ox, oy, oz, w = (np.zeros(self.nv) for _ in range(4))
        lib().orc_get_quadrature(self.h, _p(ox), _p(oy), _p(oz), _p(w))
        return ox, oy, oz, w

    def counters(self) -> dict:
        a = (ctypes.c_int64 * 13)()
        lib().orc_get_counters(self.h, a)
        keys = ("steps", "si_total", "sweeps_total", "nonconv", "fallbacks", "ig_updates",
                "pc_updates", "n0", "n1", "flag_ig", "flag_pc", "rank_ig", "rank_pc")
        return dict(zip(keys, list(a)))

    def levels(self):
        """Per correction level: flag, N_k, rank, updates."""
        a = (ctypes.c_int64 * 16)()
        L = lib().orc_get_levels(self.h, a)
        return [dict(flag=int(a[4 * k]), n=int(a[4 * k + 1]), rank=int(a[4 * k + 2]),
                     updates=int(a[4 * k + 3])) for k in range(L)]

    def history(self):
        n = self.counters()["steps"]
        arr = (StepRec * max(n, 1))()
        m = lib().orc_get_history(self.h, arr, n)
        keys = [k for k, _ in StepRec._fields_]
        return {k: np.array([getattr(arr[i], k) for i in range(m)]) for k in keys}

    def step_vectors(self) -> dict:
        """rho^{(0)}, rho^{(1/2)}, the ROM correction delta rho^{(1)}_DMD (zero
        unless applied), b~^{n-1} and whether the correction was applied, for
        the last step."""
        v = [np.zeros(self.nc) for _ in range(4)]
        used = lib().orc_get_step_vectors(self.h, *(_p(a) for a in v))
        return dict(rho0=v[0], rhalf=v[1], dpc=v[2], bt_prev=v[3], used_pc=bool(used))

    def rom(self, which: str):
        """(U, S, W) of the problem's IG (``"ig"``) or PC (``"pc"``) ROM, with
        the basis and W = B V as columns."""
        z = {"ig": 0, "pc": 1}[which] if isinstance(which, str) else int(which)
        r = lib().orc_get_rom(self.h, z, _D(), _D(), _D())
        U = np.zeros((max(r, 1), self.nc))
        Wm = np.zeros((max(r, 1), self.nc))
        S = np.zeros(max(r, 1))
        lib().orc_get_rom(self.h, z, _p(U), _p(S), _p(Wm))
        return U[:r].T.copy(), S[:r].copy(), Wm[:r].T.copy()

    def set_inflow(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().orc_set_inflow(self.h, _p(g))

    def apply_TSs(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.zeros(self.nc)
        lib().orc_apply_TSs(self.h, _p(rho), _p(out))
        return out

    def dsa_inverse(self, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        out = np.zeros(self.nc)
        lib().orc_dsa_apply_inverse(self.h, _p(rhs), _p(out))
        return out

    def dsa_matrix(self):
        n = self.nc
        bw = 3 if self.spec.scheme == "dg1" else self.spec.nx
        C = np.zeros((n, n))
        for r in range(n):
            for c in range(max(0, r - bw), min(n, r + bw + 1)):
                C[r, c] = lib().orc_dsa_entry(self.h, r, c)
        return C

    def sweep(self, j: int, s, zero_inflow: bool = False):
        s = np.ascontiguousarray(s, dtype=np.float64)
        out = np.zeros(self.nc)
        lib().orc_sweep(self.h, j, _p(s), int(zero_inflow), _p(out))
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
        except Exception:
            pass
