"""Serving (continuous batching) on the GPU, through the C ABI.

Each result must be the same alone and in the mix (bitwise: every problem has
its own state, launch shapes and fixed-order reductions), the HBM budget must
bound what is admitted at once, and a sampled request must meet the
mixed-precision bar against the FP64 oracle.
"""
import time

import numpy as np
import pytest

from paper_2603_19647_amd import rtrom
from paper_2603_19647_amd import workloads as W
from tests.gpu_util import converged_reference, mixed_bars, rel_l2, say

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(11)
    reqs = [W.serving_request(rng, i, grid=g, quad=q, nsteps=n)
            for i, (g, q, n) in enumerate([(32, (8, 4), 12), (48, (16, 4), 9), (64, (8, 4), 7),
                                            (40, (16, 8), 6)])]
    reqs.append(W.random_slab(3, 300, 16, method="rom", precision="mixed", nsteps=15))
    reqs.append(W.random_plane(4, 24, 8, 4, method="rom", precision="fp64", nsteps=10))
    reqs.append(W.random_slab(6, 200, 8, method="rom", precision="mixed", scheme="dg1", nsteps=12))
    return reqs


def _alone(spec):
    p = rtrom.Problem(spec.replace(single_wg=True))  # as the server runs it
    p.march(spec.nsteps)
    rho, st = p.rho(), p.stats()
    p.close()
    return rho, st


def test_serving_alone_equals_mix():
    reqs = _requests()
    say(f"serving mix of {len(reqs)} requests")
    alone = [_alone(s) for s in reqs]
    srv = rtrom.Server(hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        tickets = [srv.submit(s) for s in reqs]
        srv.drain()
        for s, t, (rho_a, st_a) in zip(reqs, tickets, alone):
            assert srv.poll(t) == 2  # RTROM_REQ_DONE
            rho, st, lat, mlat = srv.fetch(t)
            assert np.array_equal(rho, rho_a), s.name
            assert st["si_iters_total"] == st_a["si_iters_total"]
            assert st["steps"] == s.nsteps
            assert lat.shape == (s.nsteps,) and np.all(lat > 0) and mlat >= lat.sum() * 0.5
    finally:
        srv.close()


def test_serving_budget_bounds_admission():
    reqs = [W.random_plane(20 + i, 48, 16, 4, method="rom", precision="mixed", nsteps=25) for i in range(4)]
    need = max(rtrom.estimate_bytes(s) for s in reqs) + 25 * 64
    budget = int(need * 1.5)  # room for one request at a time, not two
    say(f"serving budget {budget} B for requests of ~{need} B")
    srv = rtrom.Server(hbm_budget_bytes=budget, max_slots=4)
    try:
        tickets = [srv.submit(s) for s in reqs]
        most = 0
        t_end = time.time() + 100
        while time.time() < t_end:
            states = [srv.poll(t) for t in tickets]
            most = max(most, sum(1 for x in states if x == 1))
            if all(x >= 2 for x in states):
                break
            time.sleep(0.001)
        srv.drain()
        assert most <= 1, most
        for s, t in zip(reqs, tickets):
            rho, st, lat, mlat = srv.fetch(t)
            rho_a, _ = _alone(s)
            assert np.array_equal(rho, rho_a)
    finally:
        srv.close()


def test_serving_sampled_request_meets_mixed_bar():
    rng = np.random.default_rng(5)
    spec = W.serving_request(rng, 0, grid=64, quad=(8, 4), nsteps=10)
    say(f"serving sampled {spec.name} vs oracle")
    ref = converged_reference(spec, spec.nsteps)
    bar = mixed_bars(spec, spec.nsteps, ref)[-1]
    srv = rtrom.Server(hbm_budget_bytes=4 << 30, max_slots=2)
    try:
        t = srv.submit(spec)
        srv.drain()
        rho, st, lat, mlat = srv.fetch(t)
    finally:
        srv.close()
    assert rel_l2(rho, ref[-1]) <= bar
