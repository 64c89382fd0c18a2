"""Build the HIP library liblbm.so for gfx950 (in-tree, next to this file).

    python -m paper_2408_15654_amd.build

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm.hip")]
HEADERS = [os.path.join(CSRC, "lbm_device.h"), os.path.join(CSRC, "arena.h"),
           os.path.join(ROOT, "include", "lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# lbm.hip is compiled twice.  The second pass (LBM_F16_PART) holds only the
# float16 step kernels, built with -ffp-contract=on: a multiply and an add
# are fused only when they are one source expression, by the front end
# (llvm.fmuladd), so every inlined copy of an expression is fused the same
# way and a site's arithmetic gives the same bits in every copy of the row
# code.  Float16 storage rounds stochastically from all 32 bits of each
# value, so that is what keeps its results independent of the tile height.
# (The back-end fusion across statements that the default allows depends on
# the surrounding code; with it, copies of the row code differed by an ulp.)
PASSES = (("main", []), ("f16", ["-DLBM_F16_PART", "-ffp-contract=on"]))


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for tag, extra in PASSES:
            obj = os.path.join(d, f"lbm_{tag}.o")
            cmd = [HIPCC, *FLAGS, *extra, "-c", "-o", obj, *SOURCES]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), cmd))
            objs.append(obj)
        for proc, cmd in procs:
            if proc.wait() != 0:
                raise subprocess.CalledProcessError(proc.returncode, cmd)
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(s) <= t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
