"""Pins of the oracle's variants beyond the paper's default configuration:

* the McClarren-Haut preconditioner (Sec. 3.3: DMD of the sweep operator
  from the iterates of one time step) alone and as the replacement of DSA in
  the ROM method (the hybrid of Sec. 4.5);
* sequential correction ROMs for iterations l >= 2 (Sec. 3.2, key feature 1:
  the ROM of iteration l is built after those of the initial guess and of
  iterations 1..l-1);
* BDF2 time stepping (Sec. 2.1 names BDF as the alternative to backward
  Euler), started with one backward-Euler step.

Each is checked against what the mathematics fixes independently of the
oracle's arithmetic: the ideal correction equation (eq. ideal_correct) for
full-span data and finite termination on a tiny grid, the fixed point of
eq. implicit_linear_system_rho (every preconditioner reaches the same
solution), Galerkin identities of the correction ROMs assembled from dense
sweeps of unit vectors, the BDF2 recurrence of an infinite medium, a dense
solve of the full BDF2 system, second-order convergence in time and particle
balance.
"""
import numpy as np
import pytest

import oracle
from paper_2603_19647_amd import workloads as W


# --------------------------------------------------------------------------
# McClarren-Haut model
# --------------------------------------------------------------------------

def _random_contraction(n, seed, rho=0.9):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return rho * A / np.abs(np.linalg.eigvals(A)).max()


def test_mh_full_span_gives_ideal_correction():
    """With n independent pairs (x, A x) the model holds A on the whole space,
    so the correction solves (I - A) d = A r exactly (eq. ideal_correct)."""
    n = 10
    A = _random_contraction(n, 1)
    rng = np.random.default_rng(2)
    M = oracle.MhModel(n, 16)
    for _ in range(n):
        x = rng.standard_normal(n)
        assert M.push(x, A @ x)
    assert M.size == n
    r = rng.standard_normal(n)
    d, ok = M.correct(r)
    assert ok
    ref = np.linalg.solve(np.eye(n) - A, A @ r)
    np.testing.assert_allclose(d, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_mh_partial_span_is_galerkin_on_the_pairs():
    """With m < n pairs the correction is the ideal correction restricted to
    span(X): Q (I - Q^T A Q)^{-1} Q^T A Q Q^T r, Q from numpy's QR of X; it is
    invariant to the scale of each pair and to the order-preserving sign
    choices of the factorisation."""
    n, m = 12, 5
    A = _random_contraction(n, 3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, m))
    M1, M2 = oracle.MhModel(n, 16), oracle.MhModel(n, 16)
    for k in range(m):
        M1.push(X[:, k], A @ X[:, k])
        s = 10.0 ** rng.uniform(-6, 6)
        M2.push(s * X[:, k], s * (A @ X[:, k]))
    r = rng.standard_normal(n)
    d1, _ = M1.correct(r)
    d2, _ = M2.correct(r)
    Q, _ = np.linalg.qr(X)
    Ar = Q.T @ A @ Q
    ref = Q @ np.linalg.solve(np.eye(m) - Ar, Ar @ (Q.T @ r))
    np.testing.assert_allclose(d1, ref, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(d2, ref, rtol=1e-9, atol=1e-12)


def test_mh_dependent_pair_skipped_and_restart_at_capacity():
    n = 8
    A = _random_contraction(n, 5)
    rng = np.random.default_rng(6)
    M = oracle.MhModel(n, 3)
    x1, x2 = rng.standard_normal(n), rng.standard_normal(n)
    assert M.push(x1, A @ x1) and M.push(x2, A @ x2)
    x3 = 2.0 * x1 - 0.5 * x2  # in span: adds nothing
    assert not M.push(x3, A @ x3)
    assert M.size == 2
    x4 = rng.standard_normal(n)
    assert M.push(x4, A @ x4) and M.size == 3
    x5 = rng.standard_normal(n)
    assert M.push(x5, A @ x5) and M.size == 1  # full: restarts from the new pair
    empty = oracle.MhModel(n, 3)
    d, ok = empty.correct(rng.standard_normal(n))
    assert not ok and not d.any()


def test_mh_finite_termination_on_tiny_slab():
    """4 cells: after at most 4 independent pairs the model is the sweep
    operator itself, the correction is exact and the next sweep passes the
    stop test, so no step needs more than N_c + 2 sweeps -- where plain SI
    (c ~ 0.98 per sweep at this optical thickness) does not converge in 60."""
    sp = W.slab(4, 8, 50.0, 0.01, 1.0, dt=1.0, tol=1e-12, max_iter=60, nsteps=5)
    mh = oracle.OracleProblem(sp.replace(method="si_dsa", precond="mh"))
    assert mh.march(5) == 0
    assert mh.history()["iters"].max() <= 4 + 2
    si = oracle.OracleProblem(sp.replace(method="si"))
    si.march(5)
    assert si.counters()["nonconv"] == 5


def _march(sp, n, **kw):
    o = oracle.OracleProblem(sp.replace(**kw))
    rhos = []
    for _ in range(n):
        o.step()
        rhos.append(o.rho())
    return o, np.array(rhos)


@pytest.mark.parametrize("kw", [dict(method="si_dsa", precond="mh"), dict(method="rom", precond="mh"),
                                dict(method="rom", pc_levels=2), dict(method="rom", pc_levels=3)],
                         ids=["mh", "hybrid_mh", "levels2", "levels3"])
def test_variants_reach_the_si_dsa_solution_every_step(kw):
    """Every preconditioner changes the iterates, never the fixed point of
    eq. implicit_linear_system_rho: at tol 1e-12 each step agrees with SI-DSA
    to the SI tolerance (the paper's own check, P:Sec. 4)."""
    sp = W.slab_two_region(nx=64, nsteps=40).replace(tol=1e-12)
    _, ref = _march(sp, 40, method="si_dsa")
    o, got = _march(sp, 40, **kw)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-9, err.max()
    assert o.counters()["nonconv"] == 0


def test_mh_accelerates_plain_si_and_hybrid_beats_mh():
    """Qualitative (the paper's Fig. for Sec. 4.5 only): McClarren-Haut needs
    far fewer sweeps than SI; the ROM initial guess and first correction cut
    them further."""
    sp = W.slab_two_region(nx=64, nsteps=40)
    it = {}
    for name, kw in (("si", dict(method="si")), ("mh", dict(method="si_dsa", precond="mh")),
                     ("hyb", dict(method="rom", precond="mh"))):
        o, _ = _march(sp, 40, **kw)
        it[name] = o.history()["iters"].mean()
    assert it["mh"] < 0.5 * it["si"]
    assert it["hyb"] < it["mh"]


# --------------------------------------------------------------------------
# Sequential correction ROMs
# --------------------------------------------------------------------------

def _dense_K(o, n):
    return np.column_stack([o.apply_TSs(np.eye(n)[:, k]) for k in range(n)])


def test_default_is_one_level():
    sp = W.slab_two_region(nx=64, nsteps=30).replace(method="rom")
    a, ra = _march(sp, 30)
    b, rb = _march(sp, 30, pc_levels=1)
    np.testing.assert_array_equal(ra, rb)
    for k in ("iters", "phase", "rank_pc", "pc_update"):
        np.testing.assert_array_equal(a.history()[k], b.history()[k])


def test_level_two_rom_is_galerkin_projection_of_ideal_correction():
    """The pairs of iteration 2, x = rho^n - rho^{(3/2)} and b = rho^{(3/2)} -
    rho^{(1)}, satisfy the same ideal correction equation C~ x = b
    (eq. ideal_correct with l = 2), so once level 2 is complete (untruncated)
    its reduced operator is dU2^T C~ dU2, C~ = (T Sigma_s)^{-1}(I - T Sigma_s)
    assembled from sweeps of unit vectors.  Column j of the difference is
    O(tol ||rho|| / dS_j) (the SI error of rho^n, not amplified by C~)."""
    sp = W.random_slab(31, 24, 8, tol=1e-13, dt=0.02, method="rom", eps_ig=1e-9, eps_pc=1e-6,
                       eps_up=1e-9, pc_levels=2)
    sp = sp.replace(sigma_s=np.maximum(sp.sigma_s, 0.5))
    o = oracle.OracleProblem(sp)
    for _ in range(400):
        if o.levels()[1]["flag"]:
            break
        o.step()
    lv = o.levels()
    assert lv[0]["flag"] and lv[1]["flag"] and lv[1]["n"] >= 2, lv
    U, S, Wm = o.rom(2)
    assert U.shape[1] == lv[1]["rank"] >= 2
    n = sp.nx
    K = _dense_K(o, n)
    Ct = np.linalg.solve(K, np.eye(n) - K)
    Cr = U.T @ Wm / S
    G = U.T @ Ct @ U
    scaled = np.linalg.norm(Cr - G, axis=0) * S / (sp.tol * np.linalg.norm(o.rho()))
    assert scaled.max() < 5.0, scaled


def test_levels_complete_in_order():
    """Phases 1..L+2: each ROM is completed after the ones before it (N0, then
    N1, N2 ...), a level's updates start only after the level below it is
    complete, ranks stay within r_max."""
    sp = W.random_slab(32, 48, 8, tol=1e-12, dt=0.02, method="rom", eps_ig=1e-9, eps_pc=1e-4,
                       eps_up=1e-9, pc_levels=2, r_max=8)
    sp = sp.replace(sigma_s=np.maximum(sp.sigma_s, 0.5))
    o = oracle.OracleProblem(sp)
    o.march(150)
    h = o.history()
    lv = o.levels()
    c = o.counters()
    assert c["flag_ig"] and lv[0]["flag"] and lv[1]["flag"], (c, lv)
    ph = h["phase"]
    assert (np.diff(ph) >= 0).all() and ph.max() == 4
    n0, n1, n2 = c["n0"], lv[0]["n"], lv[1]["n"]
    assert n0 > 0 and n1 > 0 and n2 > 0
    # phase k+1 starts the step after ROM k completes
    assert (ph[:n0] == 1).all() and (ph[n0:n0 + n1] == 2).all() and (ph[n0 + n1:n0 + n1 + n2] == 3).all()
    assert (ph[n0 + n1 + n2:] == 4).all()
    assert max(lv[0]["rank"], lv[1]["rank"], c["rank_ig"]) <= 8


# --------------------------------------------------------------------------
# BDF2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [1, 2])
def test_bdf2_infinite_medium_recurrence(dim):
    """Uniform f0 = 1, G = 0, inflow set to the uniform solution: the upwind
    differences vanish and f = u_n with u_1 = u_0 / (1 + dt sigma_a) (the
    backward-Euler start) and (3 u_n - 4 u_{n-1} + u_{n-2}) / (2 dt) +
    sigma_a u_n = 0 afterwards."""
    sa, dt = 0.7, 0.2
    sp = W.infinite_medium(dim=dim, n=12 if dim == 1 else 6, n_polar=4, n_azim=4, sigma_a=sa,
                           dt=dt, tol=1e-12).replace(time_scheme="bdf2")
    o = oracle.OracleProblem(sp)
    u = [1.0, 1.0 / (1.0 + dt * sa)]
    for n in range(1, 7):
        o.step()
        np.testing.assert_allclose(o.rho(), u[n], rtol=1e-10)
        np.testing.assert_allclose(o.f(), u[n], rtol=1e-10)
        u.append((4.0 * u[n] - u[n - 1]) / (3.0 + 2.0 * dt * sa))
        o.set_inflow([u[n + 1]] * 4)


def _dense_step_1d(sp, mu, w, fprev, fprev2, bdf2):
    nx, nv = sp.nx, len(mu)
    h = sp.lx / nx
    N = nx * nv
    A = np.zeros((N, N))
    b = np.zeros(N)
    st = sp.sigma_s + sp.sigma_a
    for j in range(nv):
        m = abs(mu[j]) / h
        for i in range(nx):
            r = j * nx + i
            A[r, r] += (1.5 if bdf2 else 1.0) / sp.dt + st[i] + m
            up = i - 1 if mu[j] > 0 else i + 1
            if 0 <= up < nx:
                A[r, j * nx + up] -= m
            else:
                b[r] += m * (sp.inflow[0] if mu[j] > 0 else sp.inflow[1])
            for k in range(nv):
                A[r, k * nx + i] -= sp.sigma_s[i] * w[k]
            hist = (2.0 * fprev[j, i] - 0.5 * fprev2[j, i]) / sp.dt if bdf2 else fprev[j, i] / sp.dt
            b[r] += hist + sp.source[i]
    return np.linalg.solve(A, b).reshape(nv, nx)


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
def test_bdf2_dense_1d(method):
    """The full (N_c N_v)^2 BDF2 system, assembled and solved densely each
    step (backward Euler for the first)."""
    sp = W.random_slab(7, 16, 4, inflow=(1.0, 0.3, 0, 0), dt=0.05, tol=1e-12, method=method,
                       time_scheme="bdf2")
    o = oracle.OracleProblem(sp)
    mu, _, _, w = o.quadrature()
    f2, f = np.zeros((4, 16)), np.zeros((4, 16))
    for n in range(1, 7):
        o.step()
        f2, f = f, _dense_step_1d(sp, mu, w, f, f2, n >= 2)
        np.testing.assert_allclose(o.rho(), w @ f, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(o.f(), f, rtol=1e-9, atol=1e-12)


def test_bdf2_second_order_backward_euler_first_order():
    """Errors at a fixed time against a fine-step reference of the same
    spatial scheme: halving dt divides the BDF2 error by ~4 and the backward
    Euler error by ~2."""
    base = W.slab(32, 8, 1.0, 0.5, 1.0, tol=1e-13, method="si_dsa")
    T = 0.4

    def run(dt, scheme):
        o = oracle.OracleProblem(base.replace(dt=dt, time_scheme=scheme))
        o.march(int(round(T / dt)))
        return o.rho()

    ref = run(0.0125 / 16, "bdf2")
    for scheme, lo, hi in (("bdf2", 1.85, 2.3), ("be", 0.85, 1.2)):
        e = [np.linalg.norm(run(dt, scheme) - ref) for dt in (0.05, 0.025, 0.0125)]
        orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert (orders > lo).all() and (orders < hi).all(), (scheme, orders)


def test_bdf2_particle_balance():
    """Per step: sum_i h [(3 rb^n - 4 rb^{n-1} + rb^{n-2}) / (2 dt) + sigma_a rb^n
    - G] + J_out - J_in = sum_i h sigma_s (rho^n - rb^n), rb = sum_j w_j f_j."""
    sp = W.random_slab(5, 64, 8, inflow=(0.7, 0.2, 0, 0), dt=0.05, time_scheme="bdf2", tol=1e-10)
    o = oracle.OracleProblem(sp)
    mu, _, _, w = o.quadrature()
    h = 1.0 / sp.nx
    hist = [w @ o.f()]
    for n in range(1, 6):
        o.step()
        f = o.f()
        rb = w @ f
        rho = o.rho()
        pos = mu > 0
        jout = (w[pos] * mu[pos] * f[pos, -1]).sum() + (w[~pos] * -mu[~pos] * f[~pos, 0]).sum()
        jin = (w[pos] * mu[pos]).sum() * 0.7 + (w[~pos] * -mu[~pos]).sum() * 0.2
        ddt = (rb - hist[-1]) / sp.dt if n == 1 else (3 * rb - 4 * hist[-1] + hist[-2]) / (2 * sp.dt)
        lhs = (h * (ddt + sp.sigma_a * rb - sp.source)).sum() + jout - jin
        rhs = (h * sp.sigma_s * (rho - rb)).sum()
        assert abs(lhs - rhs) < 1e-11 * max(1.0, np.abs(rb).sum() * h / sp.dt)
        hist.append(rb)


def test_bdf2_rom_skips_the_start_step_and_matches_si_dsa():
    sp = W.slab_two_region(nx=64, nsteps=40).replace(tol=1e-12, time_scheme="bdf2")
    _, ref = _march(sp, 40, method="si_dsa")
    o, got = _march(sp, 40, method="rom")
    h = o.history()
    assert h["ig_update"][0] == 0 and h["ig_update"][1] == 1
    assert h["phase"].max() == 3
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-9


def _dense_step_2d(sp, ox, oy, w, fprev, fprev2, bdf2):
    """The full X-Y upwind system of one step, assembled cell by cell from the
    finite-volume balance of each ordinate and solved densely."""
    n, nv = sp.nx, len(w)
    h = sp.lx / n
    N = n * n * nv
    A = np.zeros((N, N))
    b = np.zeros(N)
    st = sp.sigma_s + sp.sigma_a
    g = sp.inflow
    for j in range(nv):
        mx, my = abs(ox[j]) / h, abs(oy[j]) / h
        sx, sy = (1 if ox[j] > 0 else -1), (1 if oy[j] > 0 else -1)
        for iy in range(n):
            for ix in range(n):
                c = iy * n + ix
                r = j * n * n + c
                A[r, r] += (1.5 if bdf2 else 1.0) / sp.dt + st[c] + mx + my
                ux, uy = ix - sx, iy - sy
                if 0 <= ux < n:
                    A[r, j * n * n + iy * n + ux] -= mx
                else:
                    b[r] += mx * (g[0] if sx > 0 else g[1])
                if 0 <= uy < n:
                    A[r, j * n * n + uy * n + ix] -= my
                else:
                    b[r] += my * (g[2] if sy > 0 else g[3])
                for k in range(nv):
                    A[r, k * n * n + c] -= sp.sigma_s[c] * w[k]
                hist = (2.0 * fprev[j, c] - 0.5 * fprev2[j, c]) / sp.dt if bdf2 else fprev[j, c] / sp.dt
                b[r] += hist + sp.source[c]
    return np.linalg.solve(A, b).reshape(nv, n * n)


@pytest.mark.parametrize("method", ["si_dsa", "rom"])
def test_bdf2_dense_2d(method):
    """On an X-Y grid: the full (N_c N_v)^2 BDF2 system (Sec. 2.1's BDF
    alternative, (3 f^n - 4 f^{n-1} + f^{n-2}) / (2 dt)) assembled and solved
    densely each step, backward Euler for the first; the oracle's rho and f
    match it at every step, for both methods."""
    sp = W.random_plane(8, 6, 4, 2, inflow=(0.5, 0.0, 0.2, 0.1), dt=0.05, tol=1e-12, method=method,
                        time_scheme="bdf2")
    o = oracle.OracleProblem(sp)
    ox, oy, _, w = o.quadrature()
    nv = len(w)
    f2, f = np.zeros((nv, 36)), np.zeros((nv, 36))
    for n in range(1, 7):
        o.step()
        f2, f = f, _dense_step_2d(sp, ox, oy, w, f, f2, n >= 2)
        np.testing.assert_allclose(o.rho(), w @ f, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(o.f(), f, rtol=1e-9, atol=1e-12)
