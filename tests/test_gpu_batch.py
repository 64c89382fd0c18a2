"""Batches (through the C ABI): each simulation of a batch gives exactly
(bitwise) what it gives on its own with lbm_step, whatever else the batch
holds, whatever the schedule, across replays of the captured graphs with
host work in between, and when it joins while others are running."""
import numpy as np
import pytest

from paper_2408_15654_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("phi", "psi", "ux", "uy", "P")


def mixed_problems():
    """Different sizes, precisions, r (kernel variants), walls, density
    contrast, and step counts."""
    out = []
    specs = [
        (0, 70, 33, True, 1.0, "fp32", 41),
        (1, 61, 29, False, 0.0, "fp32", 64),
        (2, 128, 64, True, 2.0, "fp16dev", 50),
        (3, 45, 45, False, 1.0, "fp64", 23),
        (4, 200, 17, False, 0.5, "fp32", 7),
        (5, 121, 62, True, 1.0, "fp16dev", 64),
    ]
    for seed, nx, ny, walls, r, prec, steps in specs:
        pr = W.random_small(300 + seed, nx=nx, ny=ny, walls=walls, r=r, precision=prec,
                            steps=steps)
        out.append((dict(pr.params, precision=prec), pr.fields0, steps))
    rng = np.random.default_rng(7)
    pr = W.c4_instance(rng, precision="fp32", steps=64)
    out.append((pr.params, pr.fields0, 64))
    pr = W.e2_convection(nx=64, R=12.0, precision="fp32", steps=48)  # prescribed velocity
    out.append((pr.params, pr.fields0, 48))
    return out


def alone(params, fields, steps):
    sim = lbm.Simulation(params)
    sim.init_fields(*fields)
    sim.step(steps)
    out = sim.read_fields()
    sim.close()
    return out


def assert_same(a, b, label):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (label, k, float(np.abs(a[k] - b[k]).max()))


def budget_for(problems, extra=0):
    n = len(problems) + extra
    return lbm.Batch.overhead_bytes(16) + sum(lbm.Batch.instance_bytes(p) for p, _, _ in problems) \
        + (1 << 22) + n * 4096


def test_batch_equals_alone_bitwise_across_replays():
    probs = mixed_problems()
    b = lbm.Batch(budget_for(probs), max_instances=16)
    b.set_schedule(rows=0, grid_waves=0, chunk=8)
    ids = [b.submit(p, *f, n) for p, f, n in probs]
    done = 0
    for rep in range(8):  # 8 replays of 8-step graphs, host reads in between
        b.step(8)
        done += 8
        i = rep % len(ids)
        p, f, n = probs[i]
        got = b.read_fields(ids[i])
        want = alone(p, f, min(n, done))
        assert_same(got, want, f"replay {rep} sim {i}")
    for i, (p, f, n) in enumerate(probs):
        assert b.remaining(ids[i]) == 0
        assert_same(b.read_fields(ids[i]), alone(p, f, n), f"final sim {i}")
        assert b.moments(ids[i])["step"] == n
    b.close()


@pytest.mark.parametrize("rows,grid_waves,chunk", [(4, 1024, 16), (16, 0, 5), (3, 64, 1)])
def test_schedule_does_not_change_results(rows, grid_waves, chunk):
    probs = mixed_problems()[:4]
    b = lbm.Batch(budget_for(probs), max_instances=16)
    b.set_schedule(rows=rows, grid_waves=grid_waves, chunk=chunk)
    ids = [b.submit(p, *f, n) for p, f, n in probs]
    b.step(100)
    for i, (p, f, n) in enumerate(probs):
        assert_same(b.read_fields(ids[i]), alone(p, f, n), f"sched {rows},{grid_waves} sim {i}")
    b.close()


def test_admission_by_budget_and_joining_mid_run():
    probs = mixed_problems()
    big = max(lbm.Batch.instance_bytes(p) for p, _, _ in probs)
    # room for the metadata, the tile list and about two of the largest
    budget = lbm.Batch.overhead_bytes(8) + (1 << 20) + 2 * big + big // 2
    b = lbm.Batch(budget, max_instances=8)
    b.set_schedule(chunk=4)
    admitted, waiting = {}, list(range(len(probs)))
    stepped = {}
    rounds = 0
    while waiting or admitted:
        rounds += 1
        assert rounds < 200
        for i in list(waiting):  # admit what fits now
            p, f, n = probs[i]
            sid = b.try_submit(p, *f, n)
            if sid is None:
                continue
            admitted[i] = sid
            waiting.remove(i)
        assert admitted, "nothing fits an empty batch"
        b.step(4)
        for i, sid in list(admitted.items()):
            if b.remaining(sid) == 0:
                p, f, n = probs[i]
                assert_same(b.read_fields(sid), alone(p, f, n), f"joined sim {i}")
                b.retire(sid)
                del admitted[i]
                stepped[i] = True
    assert len(stepped) == len(probs)
    assert b.free_bytes() >= budget - lbm.Batch.overhead_bytes(8) - (1 << 20) - 4096
    b.close()


def test_remaining_and_stepping_past_the_end():
    p, f, _ = mixed_problems()[0]
    b = lbm.Batch(budget_for([(p, f, 5)]), max_instances=4)
    sid = b.submit(p, *f, 5)
    assert b.remaining(sid) == 5
    b.step(3)
    assert b.remaining(sid) == 2
    b.step(100)  # only 2 more are taken
    assert b.remaining(sid) == 0
    assert b.moments(sid)["step"] == 5
    assert_same(b.read_fields(sid), alone(p, f, 5), "past the end")
    with pytest.raises(lbm.LbmError):
        b.step(-1)
    with pytest.raises(lbm.LbmError):
        b.remaining(3)
    b.close()


def test_autotune_picks_a_valid_schedule_and_keeps_results():
    probs = mixed_problems()
    b = lbm.Batch(budget_for(probs), max_instances=16)
    ids = [b.submit(p, *f, 200) for p, f, _ in probs]
    s = b.autotune(probe_steps=4)
    assert s["rows"] in (0, 4, 8, 16) and s["grid_waves"] >= 0 and s["chunk"] >= 1
    b.step(200)
    for i, (p, f, _) in enumerate(probs):
        assert b.remaining(ids[i]) == 0
        assert_same(b.read_fields(ids[i]), alone(p, f, 200), f"tuned sim {i}")
    b.close()


@pytest.mark.parametrize("precision,nx,ny", [("fp32", 724, 362), ("fp32", 725, 362),
                                             ("fp64", 724, 362)])
def test_cache_resident_size_equals_batch(precision, nx, ny):
    """A single simulation whose step traffic fits the Infinity Cache
    (64-320 MB) steps with default stores, a batch always with non-temporal
    ones: the cache policy changes no result bit."""
    pr = W.c3_many_drops(precision=precision, nx=nx, ny=ny, ndrops=12)
    params = dict(pr.params, precision=precision)
    want = alone(params, pr.fields0, 20)
    b = lbm.Batch(budget_for([(params, None, 20)]), max_instances=4)
    i = b.submit(params, *pr.fields0, 20)
    b.step(20)
    got = b.read_fields(i)
    b.close()
    assert_same(got, want, f"{precision} {nx}x{ny}")
