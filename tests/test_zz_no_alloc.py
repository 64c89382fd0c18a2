"""lbm_moments_async: the moments entry point for callers that cannot
allocate (its read-back planes and partial sums live in the library's static
device buffer), checked against lbm_moments on consecutive calls."""
import numpy as np
import pytest

from paper_2408_15654_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu


def _check_same(sim, out):
    import torch

    torch.cuda.synchronize()
    got = dict(zip(lbm.Simulation.MOMENTS_ASYNC, out[:7].cpu().tolist()))
    want = sim.moments()  # the same kernels over the handle's own scratch
    for k in ("sum_phi", "sum_psi", "mom_x", "mom_y", "kinetic", "max_u"):
        assert got[k] == want[k], (k, got[k], want[k])
    assert got["nonfinite"] == 0.0
    return got


def test_moments_async_equals_moments_on_consecutive_calls():
    import torch

    out = torch.full((8,), np.nan, dtype=torch.float64, device="cuda:0")
    # first call: the 64x64 drop with its Marangoni flow (float64 storage)
    pr = W.c1_stationary_drop()
    a = lbm.Simulation(pr.params)
    a.init_fields(*pr.fields0)
    a.step(40)
    a.moments_async(out)
    first = _check_same(a, out)
    # second call on a smaller grid, float32 storage, density contrast, walls
    pr2 = W.random_small(7, nx=41, ny=29, walls=True, steps=30)
    b = lbm.Simulation(dict(pr2.params, precision="fp32"))
    b.init_fields(*pr2.fields0)
    b.step(pr2.steps)
    b.moments_async(out)
    second = _check_same(b, out)
    assert second["sum_phi"] != first["sum_phi"]
    # the first simulation again, after more steps: the buffer keeps nothing
    # from the previous call that matters
    a.step(10)
    a.moments_async(out)
    _check_same(a, out)
    a.close()
    b.close()


def test_moments_async_rejects_what_it_cannot_hold():
    import torch

    out = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    pr = W.c3_many_drops(precision="fp32", nx=1024, ny=513, ndrops=20)  # 525312 > 2^19 sites
    sim = lbm.Simulation(pr.params)
    sim.init_fields(*pr.fields0)
    with pytest.raises(lbm.LbmError) as e:
        sim.moments_async(out)
    assert e.value.status == lbm.LBM_EINVAL
    sim.close()
    fresh = lbm.Simulation(W.c1_stationary_drop().params)
    with pytest.raises(lbm.LbmError) as e:
        fresh.moments_async(out)  # no state yet
    assert e.value.status == lbm.LBM_ESTATE
    fresh.close()
