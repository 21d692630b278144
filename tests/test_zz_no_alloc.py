"""rtrom_march_batch_noalloc (the batch march for callers that cannot
allocate device memory) against rtrom_march_batch, through the C ABI: the
same problems marched by both give bitwise the same results, on two calls in
a row (the second with a smaller batch, so the static device scratch keeps
the first call's larger table), and the size limits are enforced."""
import numpy as np
import pytest

from paper_2603_19647_amd import rtrom
from paper_2603_19647_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _specs(k0, shapes):
    return [W.random_slab(k0 + k, nx, nv, method=m, precision=pr)
            for k, (nx, nv, m, pr) in enumerate(shapes)]


def _compare(specs, nsteps):
    a = [rtrom.Problem(s) for s in specs]
    b = [rtrom.Problem(s) for s in specs]
    rtrom.march_batch(a, nsteps)
    rtrom.march_batch_noalloc(b, nsteps)
    for s, x, y in zip(specs, a, b):
        np.testing.assert_array_equal(x.rho(), y.rho(), err_msg=s.name)
        np.testing.assert_array_equal(x.f(), y.f(), err_msg=s.name)
        np.testing.assert_array_equal(x.history()["iters"], y.history()["iters"], err_msg=s.name)
        assert x.stats()["si_iters_total"] == y.stats()["si_iters_total"]
    for p in a + b:
        p.close()


def test_noalloc_batch_equals_allocating_batch_two_calls():
    big = _specs(50, [(128, 16, "rom", "mixed"), (700, 32, "rom", "fp64"), (2048, 64, "si_dsa", "mixed"),
                      (333, 16, "si_dsa", "fp64"), (1500, 32, "rom", "mixed"), (64, 64, "rom", "fp64"),
                      (2500, 16, "rom", "mixed"), (900, 16, "rom", "mixed")])
    say("noalloc batch of 8, 30 steps")
    _compare(big, 30)
    small = _specs(70, [(400, 16, "rom", "mixed"), (1000, 32, "si_dsa", "mixed"), (256, 64, "rom", "fp64")])
    say("noalloc batch of 3, 20 steps")
    _compare(small, 20)


def test_noalloc_dg_and_variant_instances():
    """Instances of every device configuration in one allocation-free batch:
    piecewise-linear DG, McClarren-Haut, BDF2 and correction ROMs beside a
    default instance."""
    specs = [W.random_slab(95, 300, 16, method="rom", precision="mixed", scheme="dg1"),
             W.random_slab(96, 200, 8, method="rom", precision="fp64", precond="mh"),
             W.random_slab(97, 500, 32, method="rom", precision="mixed", time_scheme="bdf2"),
             W.random_slab(98, 250, 16, method="rom", precision="fp64", pc_levels=2),
             W.random_slab(99, 1024, 64, method="si_dsa", precision="mixed", scheme="dg1"),
             W.random_slab(100, 640, 16, method="rom", precision="mixed")]
    say("noalloc batch of the configurations, 25 steps")
    _compare(specs, 25)


def test_noalloc_limits():
    specs = _specs(90, [(100, 16, "si_dsa", "fp64"), (120, 16, "si_dsa", "fp64")])
    probs = [rtrom.Problem(s) for s in specs]
    # the histories hold 1024 steps from creation; the noalloc march never grows them
    with pytest.raises(rtrom.RtromError) as e:
        rtrom.march_batch_noalloc(probs, 1025)
    assert e.value.status == rtrom.EINVAL
    assert all(p.stats()["steps"] == 0 for p in probs)
    rtrom.march_batch_noalloc(probs, 3)
    assert all(p.stats()["steps"] == 3 for p in probs)
    for p in probs:
        p.close()


def test_noalloc_rejects_batches_beyond_the_scratch():
    spec = W.random_slab(3, 4, 2)
    probs = [rtrom.Problem(spec) for _ in range(1025)]
    with pytest.raises(rtrom.RtromError) as e:
        rtrom.march_batch_noalloc(probs, 1)
    assert e.value.status == rtrom.EINVAL
    rtrom.march_batch_noalloc(probs[:1024], 1)
    assert probs[0].stats()["steps"] == 1 and probs[1024].stats()["steps"] == 0
    for p in probs:
        p.close()
