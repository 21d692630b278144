"""The paper's numerical experiments (Sec. 4.1-4.4) in finite-volume form, on
the GPU against the FP64 oracle.

Each experiment runs its full march with ROM-SI-DSA in FP64 on both sides:
identical SI iteration counts, phases, ROM update steps and ranks at every
step, and rel. L2 <= 1e-10 (or 10x the method's own rounding spread where the
DMD solves amplify it past 1e-11).  Sec. 4.1 is the exception: its PC ROM's
snapshots are ~1e-9 of rho (two SI sweeps per step once the IG ROM exists),
so the eq. pc_stop ratio test at 1e-6 meets the snapshots' own rounding:
the oracle itself ends phase 2 anywhere from step N0 + 13 to N0 + 16 when
sigma_s is perturbed by up to three parts in 1e14.  There the GPU must stay
within the perturbed oracle runs' spread (1e-15 level perturbations) and its
N1 and total SI sweeps inside the band those runs span.  The GPU's SI-DSA march of the same problem
must reach the same solution (ROM and DSA only change the initial guess and
the preconditioner: Sec. 4.1 reports 1.02e-9 between the two, Sec. 4.3
1.3e-11), and the average SI sweeps per step of each phase are printed in the
layout of Tables 3 and 5.  The discretisation is upwind FV, not the paper's
DG-P1, so the counts are not expected to equal the paper's; the sweeps saved
by the ROM are checked qualitatively (fewer than SI-DSA in phase 3).
"""
import numpy as np
import pytest

import oracle
from paper_2603_19647_amd import rtrom
from paper_2603_19647_amd import workloads as W
from tests.gpu_util import assert_same_decisions, oracle_rounding_spread, rel_l2, say, step_both

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _table(spec, g_rom, g_si):
    hr, hs = g_rom.history(), g_si.history()
    pr = W.phase_sweeps(hr["phase"], hr["iters"])
    ps = W.phase_sweeps(hr["phase"], hs["iters"])  # SI-DSA over the ROM run's phase windows
    say(f"  {spec.name}: phase  steps  SI sweeps/step SI-DSA -> ROM")
    for key in (1, 2, 3, "all"):
        n, a = pr[key]
        if n:
            say(f"    {str(key):>5}  {n:5d}  {ps[key][1]:6.2f} -> {a:6.2f}")
    return pr, ps


def _run(spec, spread_steps=None):
    say(f"{spec.name}: {spec.nx}x{spec.ny} cells, {spec.nord} ordinates, {spec.nsteps} steps, ROM FP64")
    errs, o, g = step_both(spec, spec.nsteps)
    assert_same_decisions(o, g)
    if errs.max() > FP64_TOL:
        spread = oracle_rounding_spread(spec, spec.nsteps)
        assert np.all(errs <= np.maximum(FP64_TOL, 10.0 * spread)), (errs.max(), spread.max())
    gs = rtrom.Problem(spec.replace(method="si_dsa"))
    gs.march(spec.nsteps)
    d = rel_l2(g.rho(), gs.rho())
    say(f"  max rel L2 to the oracle {errs.max():.2e}; ROM vs SI-DSA at the end {d:.2e}")
    assert d <= 100 * spec.tol
    pr, ps = _table(spec, g, gs)
    st = g.stats()
    assert st["n0"] > 0
    if pr[3][0]:
        assert pr[3][1] < ps[3][1]
    return g, gs


def test_sec41_two_material_slab():
    spec = W.sec41_two_material()
    say(f"{spec.name}: {spec.nx} cells, {spec.nord} ordinates, {spec.nsteps} steps, ROM FP64")
    eps = (0.0, 1e-15, -1e-15, 3e-15, -3e-15)          # the accuracy spread
    eps_band = eps + (1e-14, -1e-14, 3e-14, -3e-14)  # the decisions' rounding band
    runs = [oracle.OracleProblem(spec.replace(sigma_s=spec.sigma_s * (1 + e))) for e in eps_band]
    g = rtrom.Problem(spec)
    errs, spread = [], []
    for _ in range(spec.nsteps):
        g.step()
        for o in runs:
            o.step()
        base = runs[0].rho()
        errs.append(rel_l2(g.rho(), base))
        spread.append(max(rel_l2(o.rho(), base) for o in runs[1:len(eps)]))
    errs, spread = np.array(errs), np.array(spread)
    assert np.all(errs <= np.maximum(FP64_TOL, 10.0 * spread)), (errs.max(), spread.max())
    hg = g.history()
    keys = ("iters", "phase", "ig_update", "pc_update", "rank_ig", "rank_pc")
    matches = [all(np.array_equal(hg[k], o.history()[k]) for k in keys) for o in runs]
    st = g.stats()
    n1s = sorted(o.counters()["n1"] for o in runs)
    tots = [int(o.history()["iters"].sum()) for o in runs]
    say(f"  max rel L2 to the oracle {errs.max():.2e} (oracle spread {spread.max():.2e}); N0 {st['n0']} N1 {st['n1']} "
        f"(oracle runs: {n1s}); SI sweeps {int(hg['iters'].sum())} (oracle runs: {sorted(set(tots))}); "
        f"decisions equal to oracle runs {matches}")
    # the end of phase 2 and the march's SI sweeps inside the band the oracle
    # itself spans under relative perturbations of sigma_s up to 3e-14 (where
    # in phase 3 a step needs a few more sweeps moves with the rounding too)
    assert st["n0"] == runs[0].counters()["n0"]
    assert any(matches) or (n1s[0] <= st["n1"] <= n1s[-1] and min(tots) <= int(hg["iters"].sum()) <= max(tots))
    gs = rtrom.Problem(spec.replace(method="si_dsa"))
    gs.march(spec.nsteps)
    d = rel_l2(g.rho(), gs.rho())
    say(f"  ROM vs SI-DSA at t = 1000: {d:.2e}")
    assert d <= 1000 * spec.tol  # see test_sec41_two_material_rom_matches_si_dsa_every_step
    pr, ps = _table(spec, g, gs)
    assert pr[3][1] < ps[3][1] and st["n1"] > 0


def test_sec42_gaussian_source():
    _run(W.sec42_gaussian_source(sigma_s=1.0, cfl=1.0))


def test_sec43_variable_scattering():
    _run(W.sec43_variable_scattering())


def test_sec44_lattice():
    g, gs = _run(W.sec44_lattice())
    assert g.stats()["n1"] > 0
