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
PRECONDS = ("dsa", "mh")        # correction where DSA would be: DSA or McClarren-Haut
TIME_SCHEMES = ("be", "bdf2")   # backward Euler or BDF2 (backward-Euler start)
SCHEMES = ("fv", "dg1")         # upwind finite volume (DG-0) or piecewise-linear upwind DG (slabs)


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
    precond: str = "dsa"
    time_scheme: str = "be"
    pc_levels: int = 1  # sequential correction ROMs for iterations 1..pc_levels
    mh_rank: int = 0  # McClarren-Haut pairs per model, 0 = r_max
    scheme: str = "fv"  # spatial discretisation: "fv" or "dg1" (two unknowns per cell)
    lu_tol: float = 0.0  # singular-pivot threshold of the reduced ROM systems (0 = 1e-14)
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


# --------------------------------------------------------------------------
# The paper's numerical experiments (Sec. 4) in finite-volume form.  Cross
# sections, sources, inflow and initial states as stated there; the paper's
# default tolerances (Sec. 4 preamble: eps_SISA 1e-11, eps_IG 1e-9, eps_PC
# 1e-6, eps_UP 1e-9) unless the experiment sets its own.  The discretisation
# is this library's (first-order upwind finite volumes), not the paper's
# DG-P1, so iteration counts are comparable in kind only.
# --------------------------------------------------------------------------

PAPER_EPS = dict(tol=1e-11, eps_ig=1e-9, eps_pc=1e-6, eps_up=1e-9)


def sec41_two_material(method: str = "rom", precision: str = "fp64", nsteps: int = 100) -> ProblemSpec:
    """Sec. 4.1: slab [0, 11], sigma_s = 0 / sigma_a = 1 on [0, 1] and
    sigma_s = 100 / sigma_a = 0 on [1, 11], inflow 5 at x = 0 (mu > 0) and 0 at
    x = 11, f0 = 0, no source, 6-point Gauss-Legendre, dx = 0.1 (110 cells),
    dt = 10, t in [0, 1000] (100 steps)."""
    nx = 110
    x = _centres(nx, 11.0)
    ss = np.where(x < 1.0, 0.0, 100.0)
    sa = np.where(x < 1.0, 1.0, 0.0)
    return slab(nx, 6, ss, sa, 0.0, lx=11.0, inflow=(5.0, 0.0, 0.0, 0.0), dt=10.0, method=method,
                precision=precision, nsteps=nsteps, name="sec41_two_material", **PAPER_EPS)


def sec42_gaussian_source(sigma_s: float = 1.0, cfl: float = 1.0, n: int = 81, n_azim: int = 40,
                          n_polar: int = 6, method: str = "rom", precision: str = "fp64",
                          nsteps: Optional[int] = None) -> ProblemSpec:
    """Sec. 4.2: [-1, 1]^2, sigma_a = 0, constant sigma_s, Gaussian source
    G = (10 / pi) exp(-100 (x^2 + y^2)), zero inflow and initial state,
    81^2 cells, CL(40, 6), dt = CFL dx, t in [0, 2.5], eps_SISA = 1e-12 (IG and
    UP 1e-9, PC 1e-6)."""
    h = 2.0 / n
    x = _centres(n, 2.0) - 1.0
    X, Y = np.meshgrid(x, x, indexing="xy")
    G = (10.0 / np.pi) * np.exp(-100.0 * (X ** 2 + Y ** 2))
    dt = cfl * h
    steps = int(np.ceil(2.5 / dt - 1e-9)) if nsteps is None else nsteps
    return plane(n, n, n_azim, n_polar, sigma_s, 0.0, G.reshape(-1), lx=2.0, ly=2.0, dt=dt, tol=1e-12,
                 eps_ig=1e-9, eps_pc=1e-6, eps_up=1e-9, method=method, precision=precision, nsteps=steps,
                 name=f"sec42_gauss_ss{sigma_s:g}_cfl{cfl:g}")


def sec43_variable_scattering(n: int = 81, n_azim: int = 40, n_polar: int = 6, method: str = "rom",
                              precision: str = "fp64", nsteps: Optional[int] = None) -> ProblemSpec:
    """Sec. 4.3: [-1, 1]^2, G = 0, zero inflow, isotropic initial state
    f0 = exp(-(x^2 + y^2) / (4 zeta^2)) / (4 pi zeta^2) with zeta = 1e-2,
    sigma_s = 99.9 c^4 (c + sqrt 2)^2 (c - sqrt 2)^2 + 0.1 for c = |x| < 1 and
    1 outside, sigma_a = 0, 81^2 cells, CL(40, 6), dt = dx, t in [0, 2.5]
    (102 steps), the default tolerances."""
    h = 2.0 / n
    x = _centres(n, 2.0) - 1.0
    X, Y = np.meshgrid(x, x, indexing="xy")
    c = np.sqrt(X ** 2 + Y ** 2)
    r2 = np.sqrt(2.0)
    ss = np.where(c < 1.0, 99.9 * c ** 4 * (c + r2) ** 2 * (c - r2) ** 2 + 0.1, 1.0)
    zeta = 1e-2
    f0 = np.exp(-(X ** 2 + Y ** 2) / (4.0 * zeta ** 2)) / (4.0 * np.pi * zeta ** 2)
    dt = h
    steps = int(np.ceil(2.5 / dt - 1e-9)) if nsteps is None else nsteps
    sp = plane(n, n, n_azim, n_polar, ss.reshape(-1), 0.0, 0.0, lx=2.0, ly=2.0, dt=dt, method=method,
               precision=precision, nsteps=steps, name="sec43_variable_scattering", **PAPER_EPS)
    return sp.replace(f0=f0.reshape(-1))


def sec44_lattice(n: int = 80, n_azim: int = 40, n_polar: int = 6, method: str = "rom",
                  precision: str = "fp64", nsteps: int = 80) -> ProblemSpec:
    """Sec. 4.4: [0, 5]^2 in unit blocks; absorbers (sigma_a, sigma_s) =
    (100, 0) on the lattice's dark blocks, scatterers (0, 1) elsewhere; source
    1 on the central block |x - 2.5|, |y - 2.5| < 0.5; zero inflow and initial
    state; 80^2 cells, CL(40, 6), dt = 1/16, 80 steps (t in [0, 5]),
    (eps_IG, eps_PC, eps_UP) = (1e-6, 1e-6, 1e-6), eps_SISA 1e-11.  The block
    pattern is a reading (the paper shows it only in a figure): the inner 3 x 3
    blocks alternate, the central one is the source and the four diagonal
    neighbours of it are absorbers."""
    x = _centres(n, 5.0)
    bx = np.minimum(x.astype(np.int64), 4)
    BX, BY = np.meshgrid(bx, bx, indexing="xy")
    inner = (BX >= 1) & (BX <= 3) & (BY >= 1) & (BY <= 3)
    absorber = inner & ((BX + BY) % 2 == 0) & ~((BX == 2) & (BY == 2))
    ss = np.where(absorber, 0.0, 1.0)
    sa = np.where(absorber, 100.0, 0.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    G = np.where((np.abs(X - 2.5) < 0.5) & (np.abs(Y - 2.5) < 0.5), 1.0, 0.0)
    return plane(n, n, n_azim, n_polar, ss.reshape(-1), sa.reshape(-1), G.reshape(-1), lx=5.0, ly=5.0,
                 dt=1.0 / 16.0, tol=1e-11, eps_ig=1e-6, eps_pc=1e-6, eps_up=1e-6, method=method,
                 precision=precision, nsteps=nsteps, name="sec44_lattice")


def phase_sweeps(phases, iters) -> dict:
    """Average SI sweeps per step in each phase (1, 2, 3) and over the whole
    march, from per-step phase labels and SI iteration counts (the layout of
    Tables 3 and 5; bookkeeping only)."""
    phases = np.asarray(phases)
    iters = np.asarray(iters, dtype=np.float64)
    out = {}
    for ph in (1, 2, 3):
        m = phases == ph
        out[ph] = (int(m.sum()), float(iters[m].mean()) if m.any() else float("nan"))
    out["all"] = (int(len(iters)), float(iters.mean()) if len(iters) else float("nan"))
    return out
