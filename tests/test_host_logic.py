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
