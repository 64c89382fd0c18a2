"""Continuous-batching request loop over the batch runtime.

Requests (a problem: parameters, initial fields and a step count) arrive
over time.  The loop admits every waiting request that fits the batch's
workspace (its HBM budget) and a free id, advances everything on the device
in short chunks, and retires finished solves as soon as their steps are done,
so requests that arrive while others run join the batch at the next chunk.
All device work is the library's (lbm_batch_*); this module only decides
when to call it and keeps the clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import lbm


@dataclasses.dataclass
class Request:
    rid: int
    params: dict
    fields0: tuple
    steps: int
    arrival: float  # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    sites: int
    fields: dict | None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def admission_order(waiting, order: str):
    """Order in which waiting requests are offered a slot: "arrival" (first
    come, first served) or "shortest" (least work, sites x steps, first;
    ties by arrival)."""
    if order == "arrival":
        return list(waiting)
    if order == "shortest":
        return sorted(waiting, key=lambda r: (_sites(r) * r.steps, r.arrival))
    raise ValueError(f"unknown admission order {order!r}")


def within_site_cap(running_sites: int, sites: int, n_running: int, cap) -> bool:
    """A request may join unless the running solves' sites plus its own
    would exceed cap.  An empty batch always admits (so no request waits
    for ever), and cap None means no limit."""
    return cap is None or n_running == 0 or running_sites + sites <= cap


def _sites(req) -> int:
    return int(req.params["nx"]) * int(req.params["ny"])


class Server:
    """Serve a stream of requests on one GPU with one batch.

    budget_bytes       device workspace of the batch (its HBM budget)
    chunk              steps per device round between admissions and
                       retirements
    order              admission order of waiting requests, "arrival" or
                       "shortest" (admission_order)
    max_running_sites  cap on the sites of the solves running together
                       (None: only the budget limits admission).  Every
                       running solve advances one step per launch, so a
                       solve's latency is its step count times the batch's
                       step time, which grows with the sites running; once
                       the device is saturated more sites add latency and no
                       throughput.
    keep_fields        (run) read back the final fields of these request ids
                       (others are retired without a read-back of the fields)
    """

    def __init__(self, budget_bytes: int, max_instances: int = 512, chunk: int = 64,
                 schedule: dict | None = None, order: str = "arrival",
                 max_running_sites: int | None = None):
        admission_order([], order)  # validates the name
        self.batch = lbm.Batch(budget_bytes, max_instances=max_instances)
        sched = dict(rows=0, grid_waves=0, chunk=min(chunk, 64))
        if schedule:
            sched.update(schedule)
        self.batch.set_schedule(**sched)
        self.chunk = chunk
        self.order = order
        self.max_running_sites = max_running_sites

    def _wait(self):
        """Wait for the device work enqueued so far (the batch's stream)."""
        self.batch.stream.synchronize()

    def run(self, requests: list[Request], keep_fields=frozenset(), clock=time.perf_counter,
            on_admit=None) -> tuple[list[Result], dict]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque[Request] = collections.deque()
        running: dict[int, tuple[Request, float]] = {}
        results: list[Result] = []
        site_updates = 0
        peak_running = 0
        running_sites = 0
        t0 = clock()
        while pending or waiting or running:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # the next chunk of the running solves goes to the device first;
            # admissions below then overlap with it (the library copies and
            # initialises joiners on a stream of its own) and join the chunk
            # after
            stepping = bool(running)
            if stepping:
                self.batch.step(self.chunk)
            # admit in the chosen order while they fit the budget and the
            # site cap (a request that does not fit waits; others may still
            # be admitted)
            joined = {}
            for req in admission_order(waiting, self.order):
                if not within_site_cap(running_sites + sum(_sites(r) for r, _ in joined.values()),
                                       _sites(req), len(running) + len(joined),
                                       self.max_running_sites):
                    continue
                sid = self.batch.try_submit(req.params, *req.fields0, req.steps)
                if sid is None:
                    continue
                waiting.remove(req)
                joined[sid] = (req, clock() - t0)
                if on_admit:
                    on_admit(req, sid)
            if not stepping:
                if joined:  # start them at once
                    running.update(joined)
                    running_sites += sum(_sites(r) for r, _ in joined.values())
                    peak_running = max(peak_running, len(running))
                    continue
                if pending:  # idle until the next arrival
                    delay = pending[0].arrival - (clock() - t0)
                    if delay > 0:
                        time.sleep(min(delay, 0.01))
                    continue
                if waiting:
                    raise RuntimeError("a request does not fit the empty batch")
                break
            self._wait()
            finished = [sid for sid in running if self.batch.remaining(sid) == 0]
            running.update(joined)
            running_sites += sum(_sites(r) for r, _ in joined.values())
            peak_running = max(peak_running, len(running))
            for sid in finished:
                req, adm = running[sid]
                fields = self.batch.read_fields(sid) if req.rid in keep_fields else None
                self.batch.retire(sid)
                del running[sid]
                sites = _sites(req)
                running_sites -= sites
                site_updates += sites * req.steps
                results.append(Result(req.rid, req.arrival, adm, clock() - t0, req.steps, sites,
                                      fields))
        wall = clock() - t0
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        stats = {"requests": len(results), "wall_s": round(wall, 3),
                 "aggregate_MLUPS": round(site_updates / wall / 1e6, 1),
                 "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                 "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                 "latency_max_s": round(float(lat.max()), 4),
                 "peak_running": peak_running}
        return results, stats

    def close(self):
        self.batch.close()


def serving_stream(n=200, rate=None, seed=None, precision="fp32", min_side=128, max_side=1024,
                   min_steps=1000, max_steps=20000, offered_MLUPS=None):
    """Poisson stream of solves: half drop-in-shear (2:1 channel), half
    Marangoni migration (square periodic), sites log-uniform in
    [min_side^2, max_side^2], steps uniform in [min_steps, max_steps],
    Ca ~ U[0.05, 0.4], beta ~ U[0, 0.8].  The arrival rate is `rate` per
    second, or the rate at which the stream offers `offered_MLUPS`."""
    import math

    from . import workloads as W

    rng = np.random.default_rng(W.SEED_BASE + 5 if seed is None else seed)
    probs = []
    for i in range(n):
        N = math.exp(rng.uniform(math.log(min_side ** 2), math.log(max_side ** 2)))
        steps = int(rng.integers(min_steps, max_steps + 1))
        if i % 2 == 0:
            H = max(16, int(round(math.sqrt(N / 2))))
            pr = W.shear_instance(rng, H, precision=precision, steps=steps)
        else:
            pr = W.migration_instance(rng, N, precision=precision, steps=steps)
        probs.append(pr)
    work = sum(p.sites * p.steps for p in probs) / 1e6  # million site updates
    if rate is None:
        rate = n / (work / offered_MLUPS) if offered_MLUPS else 10.0
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = [Request(i, dict(p.params, precision=precision), p.fields0, p.steps, float(t[i]))
            for i, p in enumerate(probs)]
    return reqs, rate
