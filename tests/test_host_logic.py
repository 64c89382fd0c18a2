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
