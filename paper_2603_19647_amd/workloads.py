"""Seeded synthetic problem generators.

This module only draws and lays out inputs (cross sections, sources, grid and
quadrature sizes, time step, solver parameters).  It holds none of the
method's arithmetic: no quadrature, no sweep, no DSA, no ROM.  Both the HIP
library binding and the CPU oracle consume the same ``ProblemSpec`` objects,
so the two sides always see identical arrays.

Problem statement (what the arrays mean) follows the paper's model problem:
one-group, isotropically scattering, time-dependent linear RTE on a slab or an
X-Y rectangle with isotropic inflow ``g`` and isotropic initial state ``f0``
(Sec. 2, eq. rte), backward Euler with step ``dt`` (Sec. 2.1) and the solver
tolerances of Alg. 1 / Alg. 2 (eps_SISA, eps_IG, eps_PC, eps_UP, N_iter).

Material values are sampled with the midpoint rule: a cell takes the value of
the continuous field at its centre.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

METHODS = ("si_dsa", "rom", "si")
PRECISIONS = ("fp64", "mixed")


@dataclass
class ProblemSpec:
    """One time-marching problem (inputs only)."""

    dim: int
    nx: int
    ny: int
    lx: float
    ly: float
    n_polar: int  # 1D: Gauss-Legendre order; 2D: N_z of CL(N_phi, N_z)
    n_azim: int  # 1D: 1; 2D: N_phi of CL(N_phi, N_z)
    sigma_s: np.ndarray  # [ny*nx], x fastest
    sigma_a: np.ndarray
    source: np.ndarray
    f0: Optional[np.ndarray] = None  # isotropic initial state, None = 0
    inflow: Sequence[float] = (0.0, 0.0, 0.0, 0.0)  # x-lo, x-hi, y-lo, y-hi
    dt: float = 0.01
    tol: float = 1e-8
    max_iter: int = 500
    method: str = "si_dsa"
    precision: str = "fp64"
    eps_ig: float = 1e-6
    eps_pc: float = 1e-6
    eps_up: float = 1e-6
    r_max: int = 20
    abs_up_norm: bool = False
    single_wg: bool = False  # 1D: one workgroup even when marched alone (device mode only)
    nsteps: int = 1
    name: str = ""

    @property
    def ncells(self) -> int:
        return self.nx * self.ny

    @property
    def nord(self) -> int:
        return self.n_polar if self.dim == 1 else self.n_polar * self.n_azim

    @property
    def cell_angles(self) -> int:
        return self.ncells * self.nord

    def replace(self, **kw) -> "ProblemSpec":
        return dataclasses.replace(self, **kw)


def _centres(n: int, length: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def slab(nx: int, n_polar: int, sigma_s, sigma_a, source, **kw) -> ProblemSpec:
    """1D slab [0, lx] with per-cell arrays (or scalars broadcast)."""
    lx = kw.pop("lx", 1.0)

    def arr(v):
        a = np.asarray(v, dtype=np.float64)
        return np.full(nx, float(a)) if a.ndim == 0 else a.astype(np.float64).copy()

    return ProblemSpec(dim=1, nx=nx, ny=1, lx=lx, ly=1.0, n_polar=n_polar, n_azim=1,
                       sigma_s=arr(sigma_s), sigma_a=arr(sigma_a), source=arr(source), **kw)


def plane(nx: int, ny: int, n_azim: int, n_polar: int, sigma_s, sigma_a, source,
          **kw) -> ProblemSpec:
    """2D rectangle [0, lx] x [0, ly] with per-cell arrays, x fastest."""
    lx = kw.pop("lx", 1.0)
    ly = kw.pop("ly", 1.0)
    n = nx * ny

    def arr(v):
        a = np.asarray(v, dtype=np.float64)
        return np.full(n, float(a)) if a.ndim == 0 else a.reshape(-1).astype(np.float64).copy()

    return ProblemSpec(dim=2, nx=nx, ny=ny, lx=lx, ly=ly, n_polar=n_polar, n_azim=n_azim,
                       sigma_s=arr(sigma_s), sigma_a=arr(sigma_a), source=arr(source), **kw)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def slab_two_region(nx: int = 256, nsteps: int = 50) -> ProblemSpec:
    """1D slab, 256 cells, GL16; sigma_s = 100 on [0.3, 0.7] else 1,
    sigma_a = 0.1, q = 1 on [0.4, 0.6], vacuum, dt = 0.01, plain SI-DSA FP64."""
    x = _centres(nx, 1.0)
    ss = np.where((x > 0.3) & (x < 0.7), 100.0, 1.0)
    q = np.where((x > 0.4) & (x < 0.6), 1.0, 0.0)
    return slab(nx, 16, ss, 0.1, q, dt=0.01, tol=1e-8, method="si_dsa",
                precision="fp64", nsteps=nsteps, name="slab256_gl16")


def _regions(rng: np.random.Generator, nreg: int):
    """Per-region sigma_s log-uniform on [1e-2, 1e3], sigma_a uniform [0.01, 1]."""
    ss = 10.0 ** rng.uniform(-2.0, 3.0, nreg)
    sa = rng.uniform(0.01, 1.0, nreg)
    return ss, sa


def _slab_regions(nx: int, ss_reg, sa_reg, qlo: float, qhi: float):
    nreg = len(ss_reg)
    x = _centres(nx, 1.0)
    k = np.minimum((x * nreg).astype(np.int64), nreg - 1)
    q = np.where((x > qlo) & (x < qhi), 1.0, 0.0)
    return ss_reg[k].copy(), sa_reg[k].copy(), q


def slab_random_regions(seed: int = 2, nx: int = 4096, n_polar: int = 64,
                           nsteps: int = 400, method: str = "rom",
                           precision: str = "mixed") -> ProblemSpec:
    """1D slab, 4096 cells, GL64, 32 seeded regions; q = 1 on the middle 10 %;
    dt = 0.005, 400 steps; ROM-SI-DSA with rank <= 20."""
    rng = np.random.default_rng(seed)
    ss_reg, sa_reg = _regions(rng, 32)
    ss, sa, q = _slab_regions(nx, ss_reg, sa_reg, 0.45, 0.55)
    return slab(nx, n_polar, ss, sa, q, dt=0.005, tol=1e-8, method=method,
                precision=precision, r_max=20, nsteps=nsteps,
                name=f"slab{nx}_gl{n_polar}_32reg")


def checkerboard(n: int = 256, n_azim: int = 16, n_polar: int = 8, nsteps: int = 200,
                    method: str = "rom", precision: str = "mixed") -> ProblemSpec:
    """2D [0,1]^2, n x n cells, CL(16, 8) = 128 directions; 16 x 16 blocks,
    absorber blocks (sigma_a = 10, sigma_s = 0) where the block-index sum is
    odd, scatterers (sigma_s = 1, sigma_a = 0) elsewhere; q = 1 on
    [7/16, 9/16]^2; vacuum; dt = 0.01."""
    x = _centres(n, 1.0)
    bx = np.minimum((x * 16).astype(np.int64), 15)
    BX, BY = np.meshgrid(bx, bx, indexing="xy")  # [iy][ix]
    absorber = ((BX + BY) % 2) == 1
    ss = np.where(absorber, 0.0, 1.0)
    sa = np.where(absorber, 10.0, 0.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    q = np.where((X > 7 / 16) & (X < 9 / 16) & (Y > 7 / 16) & (Y < 9 / 16), 1.0, 0.0)
    return plane(n, n, n_azim, n_polar, ss, sa, q, dt=0.01, tol=1e-8, method=method,
                 precision=precision, nsteps=nsteps, name=f"checker{n}_cl{n_azim}x{n_polar}")


def slab_batch(seed: int = 4, count: int = 512, nsteps: int = 100, method: str = "rom",
             precision: str = "mixed", ncells=(128, 2048),
             nords=(16, 32, 64)) -> List[ProblemSpec]:
    """Batch of independent 1D slabs: cells uniform on {128..2048}, S_N order
    in {16, 32, 64}, 8 regions (sigma_s log-uniform [1e-2, 1e3], sigma_a
    uniform [0.01, 1]), q = 1 on [0.45, 0.55], dt = 0.01."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.integers(ncells[0], ncells[1] + 1))
        nv = int(rng.choice(np.asarray(nords)))
        ss_reg, sa_reg = _regions(rng, 8)
        ss, sa, q = _slab_regions(nx, ss_reg, sa_reg, 0.45, 0.55)
        out.append(slab(nx, nv, ss, sa, q, dt=0.01, tol=1e-8, method=method,
                        precision=precision, nsteps=nsteps, name=f"batch{k}_n{nx}_gl{nv}"))
    return out


def gaussian_random_field(rng: np.random.Generator, n: int, corr_len: float,
                          length: float = 1.0) -> np.ndarray:
    """Zero-mean, unit-variance stationary field with squared-exponential
    covariance exp(-r^2 / (2 l^2)), by spectral (FFT) synthesis on a
    2n-periodic grid cropped to n x n.  Input generation only."""
    m = 2 * n
    h = length / n
    k = 2.0 * np.pi * np.fft.fftfreq(m, d=h)
    KX, KY = np.meshgrid(k, k, indexing="xy")
    spec = np.exp(-0.5 * (corr_len ** 2) * (KX ** 2 + KY ** 2))
    noise = rng.standard_normal((m, m))
    fld = np.real(np.fft.ifft2(np.fft.fft2(noise) * np.sqrt(spec)))[:n, :n]
    fld = fld - fld.mean()
    sd = fld.std()
    return fld / sd if sd > 0 else fld


SERVING_GRIDS = (64, 96, 128, 192, 256, 384, 512)
SERVING_QUADS = ((8, 4), (16, 4), (16, 8))  # CL(N_phi, N_z): 32, 64, 128 directions


def serving_request(rng: np.random.Generator, idx: int = 0, grid: Optional[int] = None,
               quad: Optional[Sequence[int]] = None, nsteps: Optional[int] = None,
               method: str = "rom", precision: str = "mixed") -> ProblemSpec:
    """One serving request: 2D [0,1]^2, N x N cells, CL quadrature with 32-128
    directions, sigma_s = exp(Z) with Z a Gaussian random field (mean -2,
    std 2, correlation length 0.1), sigma_a = 0.1, box source q = 1 with
    centre U(0.2, 0.8)^2 and half-width U(0.025, 0.15), dt = 0.01."""
    n = int(rng.choice(np.asarray(SERVING_GRIDS))) if grid is None else int(grid)
    qi = int(rng.integers(0, len(SERVING_QUADS)))
    nphi, nz = SERVING_QUADS[qi] if quad is None else tuple(quad)
    steps = int(rng.integers(100, 501)) if nsteps is None else int(nsteps)
    z = -2.0 + 2.0 * gaussian_random_field(rng, n, 0.1)
    ss = np.exp(z).reshape(-1)
    cx, cy = rng.uniform(0.2, 0.8, 2)
    hw = rng.uniform(0.025, 0.15)
    x = _centres(n, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    q = np.where((np.abs(X - cx) < hw) & (np.abs(Y - cy) < hw), 1.0, 0.0)
    return plane(n, n, nphi, nz, ss, 0.1, q, dt=0.01, tol=1e-8, method=method,
                 precision=precision, nsteps=steps, name=f"req{idx}_n{n}_cl{nphi}x{nz}")


def serving_stream(seed: int = 5, count: int = 64, **kw) -> List[ProblemSpec]:
    rng = np.random.default_rng(seed)
    return [serving_request(rng, i, **kw) for i in range(count)]


# --------------------------------------------------------------------------
# Small problems for tests
# --------------------------------------------------------------------------

def infinite_medium(dim: int = 1, n: int = 16, n_polar: int = 4, n_azim: int = 4,
                    sigma_a: float = 0.5, sigma_s=None, dt: float = 0.1,
                    seed: int = 0, **kw) -> ProblemSpec:
    """Homogeneous absorption, f0 = 1, G = 0; the caller sets the inflow of
    each step to the spatially uniform exact solution."""
    rng = np.random.default_rng(seed)
    nc = n if dim == 1 else n * n
    ss = rng.uniform(0.0, 5.0, nc) if sigma_s is None else np.full(nc, float(sigma_s))
    one = 1.0 / (1.0 + dt * sigma_a)
    if dim == 1:
        sp = slab(n, n_polar, ss, sigma_a, 0.0, dt=dt, **kw)
    else:
        sp = plane(n, n, n_azim, n_polar, ss, sigma_a, 0.0, dt=dt, **kw)
    return sp.replace(f0=np.ones(nc), inflow=(one, one, one, one), name="infinite_medium")


def random_slab(seed: int, nx: int, n_polar: int, nreg: int = 4, **kw) -> ProblemSpec:
    rng = np.random.default_rng(seed)
    ss_reg, sa_reg = _regions(rng, nreg)
    ss, sa, q = _slab_regions(nx, ss_reg, sa_reg, 0.45, 0.55)
    kw.setdefault("dt", 0.01)
    return slab(nx, n_polar, ss, sa, q, name=f"rslab{seed}_{nx}_{n_polar}", **kw)


def random_plane(seed: int, n: int, n_azim: int, n_polar: int, **kw) -> ProblemSpec:
    rng = np.random.default_rng(seed)
    ss = np.exp(-1.0 + 1.5 * gaussian_random_field(rng, n, 0.2))
    sa = rng.uniform(0.05, 1.0)
    x = _centres(n, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    q = np.where((np.abs(X - 0.5) < 0.15) & (np.abs(Y - 0.5) < 0.15), 1.0, 0.0)
    kw.setdefault("dt", 0.01)
    return plane(n, n, n_azim, n_polar, ss.reshape(-1), sa, q.reshape(-1),
                 name=f"rplane{seed}_{n}", **kw)
