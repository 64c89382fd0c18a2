"""Host-side logic of the library that needs no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_batch_workspace_allocator(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_2408_15654_amd", "csrc"),
                           os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and "arena ok" in out.stdout, (out.returncode, out.stdout)


def test_serving_admission_order_and_site_cap():
    from types import SimpleNamespace as NS

    from paper_2408_15654_amd import serve

    def req(rid, nx, ny, steps, arrival):
        return NS(rid=rid, params={"nx": nx, "ny": ny}, steps=steps, arrival=arrival)

    w = [req(0, 100, 50, 1000, 0.0), req(1, 40, 20, 900, 0.1),
         req(2, 200, 100, 10, 0.2), req(3, 40, 20, 900, 0.05)]
    assert [r.rid for r in serve.admission_order(w, "arrival")] == [0, 1, 2, 3]
    # work = sites x steps: 5e6, 7.2e5, 2e5, 7.2e5 (ties by arrival)
    assert [r.rid for r in serve.admission_order(w, "shortest")] == [2, 3, 1, 0]
    with pytest.raises(ValueError):
        serve.admission_order(w, "random")
    assert serve.within_site_cap(0, 10 ** 9, 0, 100)      # empty batch always admits
    assert serve.within_site_cap(60, 40, 2, 100)
    assert not serve.within_site_cap(61, 40, 2, 100)
    assert serve.within_site_cap(10 ** 9, 10 ** 9, 5, None)  # no cap


class _FakeBatch:
    """Host-side stand-in for lbm.Batch: counts steps, keeps workspace in
    whole request units, and records the order of calls."""

    class _Stream:
        def __init__(self, log):
            self.log = log

        def synchronize(self):
            self.log.append("wait")

    def __init__(self, slots):
        self.slots = slots
        self.left = {}
        self.shapes = {}
        self.log = []
        self.stream = self._Stream(self.log)
        self.next_id = 0
        self.chunks = {}  # chunks each simulation took part in

    def try_submit(self, params, phi, psi, ux, uy, nsteps):
        if len(self.left) >= self.slots:
            return None
        sid = self.next_id
        self.next_id += 1
        self.left[sid] = nsteps
        self.chunks[sid] = 0
        self.shapes[sid] = (params["ny"], params["nx"])
        self.log.append(("submit", sid))
        return sid

    def step(self, n):
        self.log.append("step")
        for sid in self.left:
            if self.left[sid] > 0:
                self.chunks[sid] += 1
            self.left[sid] = max(0, self.left[sid] - n)

    def remaining(self, sid):
        return self.left[sid]

    def read_fields(self, sid):
        return {"sid": sid}

    def retire(self, sid):
        self.log.append(("retire", sid))
        del self.left[sid]
        del self.shapes[sid]


def test_serving_loop_overlaps_admission_with_the_running_chunk():
    """The request loop (serve.Server.run) with the device replaced by a
    host stand-in: every request finishes after exactly its steps; while
    solves run, each round launches their chunk before it admits joiners
    (so the library initialises joiners while the chunk runs) and waits for
    the device only after both; joiners start with the next chunk; the site
    cap holds at every admission."""
    from types import SimpleNamespace as NS

    from paper_2408_15654_amd import serve

    reqs = [NS(rid=i, params={"nx": 10 + i, "ny": 8}, fields0=(None,) * 4,
               steps=16 * (1 + i % 3), arrival=0.0) for i in range(7)]
    srv = object.__new__(serve.Server)
    srv.batch = _FakeBatch(slots=3)
    srv.chunk = 16
    srv.order = "arrival"
    srv.max_running_sites = 3 * 16 * 8
    t = [0.0]

    def clock():
        t[0] += 1e-3
        return t[0]

    results, stats = srv.run(reqs, keep_fields={0, 3}, clock=clock)
    assert stats["requests"] == len(reqs)
    assert sorted(r.rid for r in results) == list(range(len(reqs)))
    assert all(r.finished >= r.admitted >= r.arrival for r in results)
    assert {r.rid for r in results if r.fields is not None} == {0, 3}
    log = srv.batch.log
    # after the first round, every round that steps does so before its
    # admissions, and waits after them
    first_step = log.index("step")
    for i in range(first_step, len(log)):
        if log[i] == "step":
            j = i + 1
            while j < len(log) and isinstance(log[j], tuple) and log[j][0] == "submit":
                j += 1
            assert log[j] == "wait", log[i:j + 1]
    # each solve took part in exactly steps / chunk chunks
    assert sorted(srv.batch.chunks.values()) == sorted(r.steps // 16 for r in reqs)
    assert stats["peak_running"] <= 3
