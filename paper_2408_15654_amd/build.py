"""Build the HIP library liblbm.so for gfx950 (in-tree, next to this file).

    python -m paper_2408_15654_amd.build

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm.hip")]
HEADERS = [os.path.join(CSRC, "lbm_device.h"), os.path.join(CSRC, "arena.h"),
           os.path.join(ROOT, "include", "lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -ffp-contract=off: no multiply-add is fused unless written as one, so a
# site's arithmetic gives the same bits in every copy of the step kernel's
# row code (prologue, loop, last row) and the results do not depend on the
# tile height.  Float16 storage rounds stochastically from all 32 bits of
# each value, where a one-ulp difference would change the stored value.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
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
