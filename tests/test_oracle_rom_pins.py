"""Pins of the oracle's preconditioner ROM and of Alg. 2's decisions.

The initial-guess half of Alg. 2 is pinned in test_oracle_pins.py (IG
exactness, eq. dmd-operator as a Galerkin projection, iSVD vs numpy).  Here
the other half is checked against what the paper fixes independently of the
oracle's own arithmetic:

* the correction snapshots of eq. correction_snapshot satisfy the ideal
  correction equation of the first iteration (Sec. 2.3, eq. ideal_correct),
  C~ delta rho^{(1)} = rho^{(1/2)} - rho^{(0)} with C~ = (T Sigma_s)^{-1}
  (I - T Sigma_s), so the DMD operator built from them is the Galerkin
  projection dU^T C~ dU (the same argument as for eq. dmd-operator); C~ is
  assembled densely from sweeps of unit vectors;
* the ROM correction of eq. dmd-sa, the initial guess of eq. dmd-ig, both
  error indicators and every update decision of Alg. 2 are recomputed in
  numpy from the ROMs and vectors the oracle exposes, step by step;
* the phase-2 snapshot pairs, stacked, have the SVD the PC ROM holds.
"""
import numpy as np
import pytest

import oracle
from paper_2603_19647_amd import workloads as W


def _thick_slab(seed, tol, eps_ig):
    """Tiny slab with sigma_s > 0 in every cell, so T Sigma_s is invertible."""
    sp = W.random_slab(seed, 24, 8, tol=tol, dt=0.02, method="rom", eps_ig=eps_ig,
                       eps_pc=1e-6, eps_up=1e-9)
    return sp.replace(sigma_s=np.maximum(sp.sigma_s, 0.5))


def _dense_K(o, n):
    return np.column_stack([o.apply_TSs(np.eye(n)[:, k]) for k in range(n)])


@pytest.mark.parametrize("seed,tol,eps_ig", [(21, 1e-13, 1e-9), (22, 1e-14, 1e-5), (23, 1e-13, 1e-6)])
def test_pc_rom_is_galerkin_projection_of_ideal_correction(seed, tol, eps_ig):
    """eq. correction_snapshot + eq. pc_stop: at the end of phase 2 the PC ROM
    is untruncated and C~_r = dU^T dB dV dS^{-1} equals dU^T C~ dU.  The pair
    is exact up to the SI error e of rho^n, and C~ e = (I - T Sigma_s)
    (rho^{(l-1)} - rho*) is not amplified, so column j of the difference is
    O(tol ||rho|| / dS_j).  Swapping x and b in the pair misses by >= 50x
    that bound, pairing with rho^{n-1} instead of rho^{(0)}_DMD by >= 1e9x."""
    sp = _thick_slab(seed, tol, eps_ig)
    o = oracle.OracleProblem(sp)
    for _ in range(200):
        if o.counters()["flag_pc"]:
            break
        o.step()
    c = o.counters()
    assert c["flag_pc"] == 1 and c["n1"] >= 3
    U, S, Wm = o.rom("pc")
    assert U.shape[1] == c["rank_pc"] >= 3
    n = sp.nx
    K = _dense_K(o, n)
    Ct = np.linalg.solve(K, np.eye(n) - K)
    Cr = U.T @ Wm / S
    G = U.T @ Ct @ U
    rn = np.linalg.norm(o.rho())
    scaled = np.linalg.norm(Cr - G, axis=0) * S / (tol * rn)
    assert scaled.max() < 5.0, scaled


def _reduced(U, S, Wm):
    return U.T @ Wm / S


def _rom_solve(U, S, Wm, rhs):
    return U @ np.linalg.solve(_reduced(U, S, Wm), U.T @ rhs)


@pytest.mark.parametrize("abs_norm", [False, True])
def test_alg2_vectors_indicators_and_decisions(abs_norm):
    """Every step of a march through phases 1-3, recomputed in numpy from the
    ROMs held before the step and the vectors of the step:
    rho^{(0)} (Alg. 2: rho^{n-1}, or eq. dmd-ig), rho^{(1/2)} = T Sigma_s
    rho^{(0)} + b~^{n-1} (eq. SI_rho), the ROM correction (eq. dmd-sa, from
    rho^{(1/2)} - rho^{(0)}_DMD), e_IG and e_PC (normalised by ||rho^n|| or,
    with the literal absolute norm, not), and the updates of Alg. 2: IG
    snapshot in phase 1 and when e_IG > eps_UP; PC snapshot in phase 2 for
    every step with l > 1; in phase 3, PC update when l > 1 and (IG updated
    or e_PC > eps_UP or the step could not apply the ROM correction)."""
    sp = W.slab_two_region(nx=64, nsteps=60).replace(method="rom", abs_up_norm=abs_norm)
    if abs_norm:
        sp = sp.replace(eps_up=1e-6 * 10.0)  # ||rho|| ~ 10 here: same order of updates
    o = oracle.OracleProblem(sp)
    eps = sp.eps_up
    seen = set()
    for n in range(1, sp.nsteps + 1):
        c0 = o.counters()
        bt_prev, rho_prev = o.bt(), o.rho()
        ig = o.rom("ig")
        pc = o.rom("pc")
        o.step()
        rec = {k: v[-1] for k, v in o.history().items()}
        v = o.step_vectors()
        rho = o.rho()
        phase = 1 if not c0["flag_ig"] else (2 if not c0["flag_pc"] else 3)
        seen.add(phase)
        assert rec["phase"] == phase
        np.testing.assert_array_equal(v["bt_prev"], bt_prev)
        scale = 1.0 if abs_norm else 1.0 / np.linalg.norm(rho)
        # initial guess
        if phase == 1:
            np.testing.assert_array_equal(v["rho0"], rho_prev)
        else:
            ref = _rom_solve(*ig, bt_prev)
            assert np.linalg.norm(v["rho0"] - ref) <= 1e-10 * np.linalg.norm(ref)
        # first half-iterate
        rh = o.apply_TSs(v["rho0"]) + bt_prev
        np.testing.assert_allclose(v["rhalf"], rh, rtol=1e-12, atol=1e-14 * np.abs(rh).max())
        # ROM correction of the first iteration
        if phase == 3 and rec["iters"] > 1:
            assert v["used_pc"]
            ref = _rom_solve(*pc, v["rhalf"] - v["rho0"])
            assert np.linalg.norm(v["dpc"] - ref) <= 1e-9 * np.linalg.norm(ref) + 1e-300
        else:
            assert not v["used_pc"]
        # indicators and decisions
        if phase == 1:
            assert rec["e_ig"] < 0 and rec["ig_update"] == 1
            continue
        e_ig = np.linalg.norm(v["rho0"] - rho) * scale
        assert rec["e_ig"] == pytest.approx(e_ig, rel=1e-12)
        assert rec["ig_update"] == int(e_ig > eps)
        x = rho - v["rhalf"]
        if rec["iters"] == 1:
            assert rec["pc_update"] == 0 and rec["e_pc"] < 0
        elif phase == 2:
            assert rec["pc_update"] == 1 and rec["e_pc"] < 0
        else:
            e_pc = np.linalg.norm(v["dpc"] - x) * scale
            assert rec["e_pc"] == pytest.approx(e_pc, rel=1e-12)
            assert rec["pc_update"] == int(e_ig > eps or e_pc > eps)
    assert seen == {1, 2, 3}
    c = o.counters()
    assert c["n0"] > 0 and c["n1"] > 0


def test_phase2_pc_pairs_have_the_rom_svd():
    """The phase-2 snapshot pairs of eq. correction_snapshot, x = rho^n -
    rho^{(1/2)} and b = rho^{(1/2)} - rho^{(0)}_DMD, stacked into dR and dB
    over the steps with l > 1: numpy's SVD of dR gives the PC ROM's singular
    values, and (after aligning column signs) its basis and the DMD operator
    dU^T dB dV dS^{-1}."""
    sp = _thick_slab(21, 1e-13, 1e-9)
    o = oracle.OracleProblem(sp)
    X, B = [], []
    while not o.counters()["flag_pc"]:
        ph = 1 if not o.counters()["flag_ig"] else 2
        o.step()
        it = o.history()["iters"][-1]
        if ph == 2 and it > 1:
            v = o.step_vectors()
            X.append(o.rho() - v["rhalf"])
            B.append(v["rhalf"] - v["rho0"])
    dR, dB = np.array(X).T, np.array(B).T
    u, s, vt = np.linalg.svd(dR, full_matrices=False)
    U, S, Wm = o.rom("pc")
    assert len(S) == len(s)
    np.testing.assert_allclose(S, s, rtol=1e-9, atol=1e-12 * s[0])
    d = np.sign(np.sum(u * U, axis=0))
    lead = s / s[0] > 1e-6  # directions resolved well above the rounding of dR
    np.testing.assert_allclose((U * d)[:, lead], u[:, lead], atol=1e-8)
    A_ref = u.T @ dB @ vt.T / s
    A = (d[:, None] * _reduced(U, S, Wm) * d[None, :])
    k = int(lead.sum())
    np.testing.assert_allclose(A[:k, :k], A_ref[:k, :k], rtol=0, atol=1e-6 * np.abs(A_ref[:k, :k]).max())


def test_sec41_two_material_rom_matches_si_dsa_every_step():
    """Sec. 4.1 in FV form on the oracle: the ROM march passes through all
    three phases and stays on the SI-DSA solution at every step, with fewer
    sweeps.  The two differ by what the stop test leaves: at dt = 10 the
    scattering region has c = sigma_s / (sigma_s + 1/dt) = 0.999, so an
    iterate whose update is below tol can sit up to ~1/(1 - c) = 1000 times
    tol from the fixed point (the paper reports 1.02e-9 between the two
    methods at t = 1000 with the same tol = 1e-11)."""
    sp = W.sec41_two_material()
    a = oracle.OracleProblem(sp, method="si_dsa")
    b = oracle.OracleProblem(sp, method="rom")
    worst = 0.0
    for _ in range(sp.nsteps):
        a.step()
        b.step()
        worst = max(worst, np.linalg.norm(b.rho() - a.rho()) / np.linalg.norm(a.rho()))
    assert worst <= 1000 * sp.tol, worst
    assert set(b.history()["phase"]) == {1, 2, 3}
    assert b.counters()["si_total"] < a.counters()["si_total"]


@pytest.mark.parametrize("dim", [1, 2])
def test_singular_reduced_systems_fall_back_to_si_dsa(dim):
    """R17 (a reduced ROM system whose LU meets a pivot below the threshold is
    singular; the step then takes the plain initial guess and DSA for that
    ROM).  With the threshold raised so that every reduced system is
    singular, the ROM march IS the SI-DSA march: the same iterates, bitwise,
    and the same sweep counts, while its ROMs still collect snapshots, change
    phase and count a fallback on every step that had a ROM to apply."""
    if dim == 1:
        base = W.random_slab(81, 64, 8, dt=0.01, tol=1e-10, nsteps=30)
    else:
        base = W.random_plane(81, 12, 4, 2, dt=0.02, tol=1e-10, nsteps=30)
    rom = oracle.OracleProblem(base.replace(method="rom", lu_tol=10.0))
    ref = oracle.OracleProblem(base.replace(method="si_dsa"))
    for _ in range(base.nsteps):
        rom.step()
        ref.step()
        np.testing.assert_array_equal(rom.rho(), ref.rho())
    hr, hs = rom.history(), ref.history()
    np.testing.assert_array_equal(hr["iters"], hs["iters"])
    c = rom.counters()
    assert c["flag_ig"] == 1 and c["n0"] > 0, c
    # every step after N0 fell back for the IG ROM, every step after N0 + N1
    # for the PC ROM as well
    assert c["flag_pc"] == 1, c
    assert c["fallbacks"] == (base.nsteps - c["n0"]) + (base.nsteps - c["n0"] - c["n1"]), c
    assert hr["fallback"][c["n0"]:].all() and not hr["fallback"][:c["n0"]].any()
    # the same march at the default threshold uses its ROMs and differs
    plain = oracle.OracleProblem(base.replace(method="rom"))
    plain.march(base.nsteps)
    assert plain.counters()["fallbacks"] == 0
    assert plain.history()["iters"].sum() < hs["iters"].sum()
