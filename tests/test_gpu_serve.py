"""The continuous-batching request loop: requests that arrive while others
run are admitted as workspace frees up, and every result is exactly
(bitwise) what the same problem gives when solved alone."""
import numpy as np
import pytest

from paper_2408_15654_amd import lbm, serve

pytestmark = pytest.mark.gpu


def alone(req):
    sim = lbm.Simulation(req.params)
    sim.init_fields(*req.fields0)
    sim.step(req.steps)
    out = sim.read_fields()
    sim.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
def test_served_results_equal_alone_and_requests_join_mid_run(precision):
    reqs, _ = serve.serving_stream(n=10, rate=400.0, seed=11, precision=precision,
                                   min_side=48, max_side=160, min_steps=40, max_steps=300)
    biggest = max(lbm.Batch.instance_bytes(r.params) for r in reqs)
    budget = lbm.Batch.overhead_bytes(16) + (1 << 20) + 3 * biggest  # room for ~3 at a time
    srv = serve.Server(budget, max_instances=16, chunk=16)
    joins = []
    results, stats = srv.run(reqs, keep_fields={r.rid for r in reqs},
                             on_admit=lambda req, sid: joins.append(
                                 (req.rid, len(srv.batch.shapes))))
    srv.close()
    assert stats["requests"] == len(reqs)
    assert stats["peak_running"] >= 2
    # some request was admitted while at least one other was already running
    assert any(n_running > 1 for _, n_running in joins)
    by_id = {r.rid: r for r in reqs}
    for res in results:
        want = alone(by_id[res.rid])
        for k in ("phi", "psi", "ux", "uy", "P"):
            assert np.array_equal(res.fields[k], want[k]), (res.rid, k)
        assert res.finished >= res.admitted >= res.arrival - 1e-9
    assert stats["latency_p99_s"] >= stats["latency_p50_s"] > 0


def test_least_work_first_under_a_site_cap():
    """Admission by least work under a cap on the running sites: the cap
    holds at every admission (unless the batch was empty), every request
    completes, and results stay bitwise those of the solve alone."""
    reqs, _ = serve.serving_stream(n=12, rate=600.0, seed=12, precision="fp32",
                                   min_side=48, max_side=160, min_steps=40, max_steps=300)
    sizes = [int(r.params["nx"]) * int(r.params["ny"]) for r in reqs]
    cap = 2 * max(sizes)
    budget = lbm.Batch.overhead_bytes(16) + (1 << 20) + sum(
        lbm.Batch.instance_bytes(r.params) for r in reqs)  # the budget never binds
    srv = serve.Server(budget, max_instances=16, chunk=16, order="shortest",
                       max_running_sites=cap)
    over = []

    def on_admit(req, sid):
        running = sum(ny * nx for ny, nx in srv.batch.shapes.values())
        if len(srv.batch.shapes) > 1 and running > cap:
            over.append((req.rid, running))

    check = {r.rid for r in reqs[::3]}
    results, stats = srv.run(reqs, keep_fields=check, on_admit=on_admit)
    srv.close()
    assert not over
    assert stats["requests"] == len(reqs)
    by_id = {r.rid: r for r in reqs}
    for res in results:
        if res.fields is None:
            continue
        want = alone(by_id[res.rid])
        for k in ("phi", "psi", "ux", "uy", "P"):
            assert np.array_equal(res.fields[k], want[k]), (res.rid, k)
