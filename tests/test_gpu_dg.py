"""GPU parity of the piecewise-linear upwind DG scheme (eq. DG with K = 1,
Sec. 2.1) with its modified-interior-penalty DSA against the FP64 oracle,
through the C ABI, on slabs; also with McClarren-Haut (alone and in the
hybrid) and with BDF2 time stepping.

Bars as for finite volumes: FP64 runs agree with the oracle to rel. L2 <=
1e-10 at every step (cell averages and slopes, also cell by cell) with
identical SI counts, phases, ROM updates and ranks; ROM runs, whose
decisions follow rounding past some step, within 10x the oracle's own
rounding spread (two oracle runs with sigma_s scaled by 1 +- 1e-15) with
counts identical up to the first step where perturbed oracle runs disagree.
Mixed runs stay within max(1e-8, the FP64 oracle's own distance) of the
converged FP64 solution at every step.
"""
import numpy as np
import pytest

import oracle
from paper_2603_19647_amd import rtrom
from paper_2603_19647_amd import workloads as W
from tests.gpu_util import (assert_same_decisions, converged_reference, count_horizon, elementwise_err,
                            mixed_bars, oracle_rounding_spread, rel_l2, say, step_both)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _bar(spec, n):
    if spec.method != "rom":
        return FP64_TOL
    return np.maximum(FP64_TOL, 10.0 * oracle_rounding_spread(spec, n))


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
@pytest.mark.parametrize("nx,nv", [(1, 2), (2, 4), (5, 4), (64, 8), (129, 16), (300, 32), (1024, 64), (700, 256)])
def test_dg_fp64_matches_oracle(method, nx, nv):
    """Sizes across the sweep row classes (up to 16 cells per lane run), a
    ragged last run, the largest DG slab, the most ordinate pairs, and the
    degenerate slabs of one and two cells (both faces vacuum boundaries)."""
    spec = W.random_slab(70 + nx, nx, nv, dt=0.02, tol=1e-8, method=method, scheme="dg1",
                         inflow=(0.8, 0.3, 0.0, 0.0), nsteps=25)
    n = spec.nsteps
    say(f"dg fp64 {method} nx={nx} nv={nv}")
    horizon = count_horizon(spec, n) if method == "rom" else n
    errs, o, g = step_both(spec, n)
    assert (errs <= _bar(spec, n)).all(), errs.max()
    ho, hg = o.history(), g.history()
    for key in ("iters", "phase", "ig_update", "pc_update", "rank_ig", "rank_pc"):
        np.testing.assert_array_equal(hg[key][:horizon], ho[key][:horizon], err_msg=key)
    if horizon == n:
        assert_same_decisions(o, g)
    assert elementwise_err(g.rho(), o.rho()) <= 1e-8
    assert rel_l2(g.f(), o.f()) <= 1e-9
    assert rel_l2(g.rhs(), o.bt()) <= 1e-9
    assert g.rho().shape == (2 * nx,)


def test_dg_initial_state_and_rhs():
    """f0 and the right-hand side of the first step: the cell averages carry
    f0, the slopes start at zero, b~ as the oracle's."""
    spec = W.random_slab(5, 200, 16, dt=0.05, scheme="dg1", inflow=(1.0, 0.0, 0.0, 0.0))
    f0 = 0.5 + 0.25 * np.sin(np.linspace(0.0, 3.0, spec.nx))
    spec = spec.replace(f0=f0)
    say("dg initial state")
    o = oracle.OracleProblem(spec)
    g = rtrom.Problem(spec)
    np.testing.assert_array_equal(g.rho()[::2], f0)
    np.testing.assert_array_equal(g.rho()[1::2], 0.0)
    assert rel_l2(g.rhs(), o.bt()) <= 1e-13
    o.step()
    g.step()
    assert rel_l2(g.rho(), o.rho()) <= FP64_TOL


def test_dg_infinite_medium_exact_decay():
    sa, dt = 0.7, 0.2
    spec = W.infinite_medium(dim=1, n=40, n_polar=8, sigma_a=sa, dt=dt, tol=1e-12).replace(scheme="dg1")
    say("dg infinite medium")
    g = rtrom.Problem(spec)
    for n in range(1, 7):
        g.step()
        expect = (1.0 + dt * sa) ** (-n)
        np.testing.assert_allclose(g.rho()[::2], expect, rtol=1e-10)
        np.testing.assert_allclose(g.rho()[1::2], 0.0, atol=1e-12)
        g.set_inflow([(1.0 + dt * sa) ** (-(n + 1))] * 4)


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
def test_sec41_two_material_slab_dg_on_device(method):
    """The paper's Sec. 4.1 slab in its own DG-P1 form: per-step SI counts as
    the oracle's (SI-DSA: 15-31 sweeps per step; the ROM method 2-5 on
    average in phase 3) and the same solution.  Nearly steady (dt = 10) and
    optically thick, this setup amplifies rounding: the correction ROM's
    rank at the start of phase 3 flips, and with it the counts of the
    following steps, when sigma_s is scaled by 1 +- 1e-11 in the oracle
    itself (the device, whose sums run in another order, takes the counts
    of such a run).  Counts are compared up to the first step where such
    oracle runs disagree."""
    spec = W.sec41_two_material(method=method).replace(scheme="dg1")
    n = spec.nsteps
    say(f"sec41 dg {method}")
    horizon = count_horizon(spec, n, eps=(1e-15, -1e-15, 1e-13, 1e-11, -1e-11)) if method == "rom" else n
    say(f"  count horizon {horizon}")
    errs, o, g = step_both(spec, n)
    assert (errs <= _bar(spec, n)).all(), errs.max()
    ho, hg = o.history(), g.history()
    np.testing.assert_array_equal(hg["iters"][:horizon], ho["iters"][:horizon])
    np.testing.assert_array_equal(hg["phase"][:horizon], ho["phase"][:horizon])
    it = hg["iters"]
    if method == "si_dsa":
        assert it.min() >= 15 and it.max() <= 31
    else:
        ph3 = hg["phase"] == 3
        assert ph3.sum() >= 50 and 2.0 <= it[ph3].mean() <= 5.0
    say(f"  sweeps per step: device {it.mean():.2f}, oracle {ho['iters'].mean():.2f}")


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
def test_dg_mixed_meets_fp64_bar(method):
    spec = W.random_slab(81, 512, 32, dt=0.01, tol=1e-8, method=method, precision="mixed", scheme="dg1",
                         inflow=(1.0, 0.0, 0.0, 0.0), nsteps=40)
    say(f"dg mixed {method}")
    ref = converged_reference(spec, spec.nsteps)
    bars = mixed_bars(spec, spec.nsteps, ref, method=method)
    g = rtrom.Problem(spec)
    for k in range(spec.nsteps):
        g.step()
        e = rel_l2(g.rho(), ref[k])
        assert e <= bars[k], (k, e, bars[k])
    assert g.stats()["nonconverged_steps"] == 0
    assert g.stats()["fp32_sweeps"] > 0


def test_dg_plain_si_matches_oracle():
    spec = W.random_slab(82, 96, 8, dt=0.05, tol=1e-10, method="si", scheme="dg1", max_iter=2000, nsteps=4)
    say("dg plain si")
    errs, o, g = step_both(spec, spec.nsteps)
    assert (errs <= FP64_TOL).all(), errs.max()
    np.testing.assert_array_equal(g.history()["iters"], o.history()["iters"])


def test_dg_correction_levels_match_oracle():
    """Sequential correction ROMs (pc_levels 2) on DG unknowns."""
    sp = W.random_slab(83, 256, 16, dt=0.02, method="rom", scheme="dg1", eps_ig=1e-9, eps_pc=1e-4,
                       eps_up=1e-9, r_max=8, tol=1e-10, pc_levels=2, nsteps=80)
    spec = sp.replace(sigma_s=np.maximum(sp.sigma_s, 0.5))
    n = spec.nsteps
    say("dg levels")
    horizon = count_horizon(spec, n)
    errs, o, g = step_both(spec, n)
    assert (errs <= _bar(spec, n)).all(), errs.max()
    ho, hg = o.history(), g.history()
    for key in ("iters", "phase", "ig_update", "pc_update", "rank_ig", "rank_pc"):
        np.testing.assert_array_equal(hg[key][:horizon], ho[key][:horizon], err_msg=key)
    assert len(g.levels()) == 2 and g.levels()[0]["flag"] == o.levels()[0]["flag"] == 1


def test_dg_batched_with_fv_bitwise():
    """A batch mixing DG and finite-volume instances (both precisions, both
    methods): every instance marches to bitwise the result it reaches alone."""
    specs = []
    for k in range(8):
        s = W.random_slab(90 + k, 64 + 113 * k, (8, 16, 32)[k % 3], dt=0.01, nsteps=20,
                          method=("rom", "si_dsa")[k % 2 == 1 and k > 4], precision=("fp64", "mixed")[(k // 2) % 2])
        specs.append(s.replace(scheme="dg1") if k % 2 == 0 else s)
    say("dg/fv batch")
    alone = []
    for s in specs:
        p = rtrom.Problem(s.replace(single_wg=True))
        p.march(s.nsteps)
        alone.append(p.rho())
        p.close()
    probs = [rtrom.Problem(s) for s in specs]
    rtrom.march_batch(probs, specs[0].nsteps)
    for a, p in zip(alone, probs):
        np.testing.assert_array_equal(p.rho(), a)
        p.close()


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
def test_dg_mcclarren_haut_fp64_matches_oracle(method):
    """McClarren-Haut on DG unknowns, alone and as the hybrid with the ROM
    method (Sec. 3.3, Sec. 4.5): per-step results within 10x the oracle's own
    rounding spread (its small reduced systems amplify rounding), counts,
    phases and ranks identical up to the first step where perturbed oracle
    runs disagree."""
    spec = W.slab_two_region(nx=128, nsteps=12).replace(scheme="dg1", method=method, precond="mh")
    n = spec.nsteps
    say(f"dg mh fp64 {method}")
    horizon = count_horizon(spec, n)
    errs, o, g = step_both(spec, n)
    bar = np.maximum(FP64_TOL, 10.0 * oracle_rounding_spread(spec, n))
    assert (errs <= bar).all(), errs.max()
    ho, hg = o.history(), g.history()
    for key in ("iters", "phase", "ig_update", "pc_update", "rank_ig", "rank_pc"):
        np.testing.assert_array_equal(hg[key][:horizon], ho[key][:horizon], err_msg=key)
    assert g.stats()["nonconverged_steps"] == 0


def test_dg_mcclarren_haut_mixed_meets_fp64_bar():
    spec = W.slab_two_region(nx=128, nsteps=20).replace(scheme="dg1", method="rom", precond="mh",
                                                        precision="mixed")
    say("dg mh mixed")
    ref = converged_reference(spec, spec.nsteps)
    bars = mixed_bars(spec, spec.nsteps, ref, method="rom")
    g = rtrom.Problem(spec)
    for k in range(spec.nsteps):
        g.step()
        e = rel_l2(g.rho(), ref[k])
        assert e <= bars[k], (k, e, bars[k])
    assert g.stats()["nonconverged_steps"] == 0


@pytest.mark.parametrize("method,nx,nv", [("si_dsa", 200, 16), ("rom", 300, 32), ("rom", 1024, 16)])
def test_dg_bdf2_fp64_matches_oracle(method, nx, nv):
    """BDF2 on DG unknowns (a backward-Euler start, then the BDF2 transport
    and DSA operators): results, f and b~ as the oracle's at every step."""
    spec = W.random_slab(60 + nx, nx, nv, dt=0.01, tol=1e-8, method=method, scheme="dg1", time_scheme="bdf2",
                         inflow=(0.8, 0.3, 0.0, 0.0), nsteps=30)
    n = spec.nsteps
    say(f"dg bdf2 fp64 {method} nx={nx} nv={nv}")
    horizon = count_horizon(spec, n) if method == "rom" else n
    errs, o, g = step_both(spec, n)
    assert (errs <= _bar(spec, n)).all(), errs.max()
    ho, hg = o.history(), g.history()
    for key in ("iters", "phase", "ig_update", "pc_update", "rank_ig", "rank_pc"):
        np.testing.assert_array_equal(hg[key][:horizon], ho[key][:horizon], err_msg=key)
    assert rel_l2(g.f(), o.f()) <= 1e-9
    assert rel_l2(g.rhs(), o.bt()) <= 1e-9


def test_dg_bdf2_infinite_medium_closed_form():
    sa, dt = 0.7, 0.2
    spec = W.infinite_medium(dim=1, n=40, n_polar=8, sigma_a=sa, dt=dt, tol=1e-12).replace(
        scheme="dg1", time_scheme="bdf2")
    say("dg bdf2 infinite medium")
    g = rtrom.Problem(spec)
    u = [1.0, 1.0 / (1.0 + dt * sa)]
    for n in range(1, 8):
        g.step()
        np.testing.assert_allclose(g.rho()[::2], u[n], rtol=1e-10)
        np.testing.assert_allclose(g.rho()[1::2], 0.0, atol=1e-12)
        u.append((4.0 * u[n] - u[n - 1]) / (3.0 + 2.0 * dt * sa))
        g.set_inflow([u[n + 1]] * 4)


def test_dg_bdf2_mixed_meets_fp64_bar():
    spec = W.random_slab(87, 400, 32, dt=0.01, tol=1e-8, method="rom", precision="mixed", scheme="dg1",
                         time_scheme="bdf2", inflow=(1.0, 0.0, 0.0, 0.0), nsteps=40)
    say("dg bdf2 mixed")
    ref = converged_reference(spec, spec.nsteps)
    bars = mixed_bars(spec, spec.nsteps, ref, method="rom")
    g = rtrom.Problem(spec)
    for k in range(spec.nsteps):
        g.step()
        e = rel_l2(g.rho(), ref[k])
        assert e <= bars[k], (k, e, bars[k])
    assert g.stats()["nonconverged_steps"] == 0


def test_dg_variants_batched_bitwise():
    """A batch of DG instances with DSA, McClarren-Haut and BDF2 beside finite
    volumes: every instance marches to bitwise the result it reaches alone."""
    kinds = [dict(), dict(precond="mh"), dict(time_scheme="bdf2"), dict(precond="mh", time_scheme="bdf2")]
    specs = []
    for k in range(8):
        s = W.random_slab(110 + k, 80 + 111 * k, (8, 16, 32)[k % 3], dt=0.01, nsteps=20, method="rom",
                          precision=("fp64", "mixed")[(k // 4) % 2])
        specs.append(s.replace(scheme="dg1", **kinds[k % 4]) if k < 6 else s.replace(**kinds[k % 4]))
    say("dg variants batch")
    alone = []
    for s in specs:
        p = rtrom.Problem(s.replace(single_wg=True))
        p.march(s.nsteps)
        alone.append(p.rho())
        p.close()
    probs = [rtrom.Problem(s) for s in specs]
    rtrom.march_batch(probs, specs[0].nsteps)
    for a, p in zip(alone, probs):
        np.testing.assert_array_equal(p.rho(), a)
        p.close()
