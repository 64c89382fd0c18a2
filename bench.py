#!/usr/bin/env python3
"""Throughput of the fused coupled three-field lattice Boltzmann step on one GPU.

Workload: the 2048x2048 periodic many-drop field (400 drops, radii U[8,24],
density and viscosity ratio 10, beta = 0.5, D = 0.01, M = 0.02, W = 4,
random divergence-free initial velocity), float32 populations.  A step is one
launch of the fused step kernel over the whole grid; inputs are resident in
HBM before timing starts.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
                    [--no-cpu-baseline] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak (AMD spec)
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16dev": 2}
FIELD_BYTES = {"fp64": 8, "fp32": 4, "fp16dev": 4}
KERNEL_SOURCES = ("paper_2408_15654_amd/csrc/lbm.hip", "paper_2408_15654_amd/csrc/lbm_device.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "lbm_step_kernel_many_drops_2048_{}_counters.txt")


def algorithmic_bytes_per_site(precision: str, has_s: bool) -> int:
    """Bytes one site-update must move: 26 live populations read and written
    (f_0..f_8, g_0..g_8, h_1..h_8) plus the previous level read and written.
    float64/float32 storage keep (phi, psi) as rest values and (ux, uy) and,
    with a density contrast, (Sx, Sy) as aux; float16 storage keeps
    (phi, psi, P, rho ux, rho uy) in float32 as rest values (the bases of the
    stored deviations) and (Sx, Sy) as aux."""
    s = 2 if has_s else 0
    fields = 5 + s if precision == "fp16dev" else 4 + s
    return 2 * 26 * STORE_BYTES[precision] + 2 * fields * FIELD_BYTES[precision]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(precision: str):
    """The committed rocprofv3 counter summary (key = value lines), or None."""
    try:
        with open(COUNTERS_FILE.format(precision)) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    out = {}
    for ln in lines:
        if "=" in ln and not ln.lstrip().startswith("#"):
            k, v = ln.split("=", 1)
            out[k.strip()] = v.strip()
    return out


def measured_traffic(sites: int, precision: str):
    """HBM bytes per launch from the committed counter summary: FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by what the same counter reads for a
    plain copy kernel of known size.  None if the summary is missing or was
    taken on a different kernel source or problem."""
    c = read_counters(precision)
    if not c or c.get("source_hash") != kernel_source_hash():
        return None
    if int(c.get("sites", -1)) != sites:
        return None
    return float(c["hbm_bytes_per_launch"])


def cpu_baseline(pr, target_seconds=15.0):
    """The FP64 oracle on the host cores on a bounded sample of the same
    workload: the same 2048x2048 problem for a few steps."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle

    sim = oracle.OracleSim(pr.params, *pr.fields0)
    t0 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(target_seconds / max(one, 1e-3))))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(pr.sites * n / dt / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"FP64 oracle, same 2048x2048 many-drop problem, {n} steps "
                      f"after 1 warm-up step ({dt:.1f} s)"}


def copy_calibration(device="cuda:0", nbytes=1 << 30):
    """A plain elementwise kernel (y = -x over float32) of known size: it
    reads and writes nbytes each.  Used to scale the HBM counters and as the
    practical bandwidth ceiling.  (A same-dtype tensor copy is a DMA transfer,
    not a kernel, and the counters do not see it.)"""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"read_bytes": nbytes, "write_bytes": nbytes, "ms": ms,
            "GBs": 2 * nbytes / ms / 1e6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp16dev"])
    ap.add_argument("--rows", type=int, default=0, help="tile height override")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2408_15654_amd import lbm, workloads

    if args.copy_calibration:
        print(json.dumps({"copy_calibration": copy_calibration()}), flush=True)
        return

    pr = workloads.c3_many_drops(precision=args.precision)
    sim = lbm.Simulation(pr.params, device="cuda:0")
    if args.rows:
        sim.set_tile_rows(args.rows)
    sim.init_fields(*pr.fields0)
    m0 = sim.moments()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = e0.elapsed_time(e1)
    m1 = sim.moments()

    sites = pr.sites
    sec = wall
    mlups = sites * args.steps / sec / 1e6
    has_s = pr.params["rhoA"] != pr.params["rhoB"]
    bps = algorithmic_bytes_per_site(args.precision, has_s)
    per_launch_ms = ms_events / args.steps
    achieved = bps * sites / (per_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(sites, args.precision)

    out = {
        "metric": "MLUPS of coupled 3-field LB step, % HBM peak; p50/p99 batched-solve latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"many_drops_2048x2048_{args.precision}", "nx": 2048,
                   "ny": 2048, "drops": 400, "density_ratio": 10, "viscosity_ratio": 10,
                   "precision": args.precision, "parallelism": "single GPU",
                   "bytes_per_site_update": bps},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": sim.step_kernel_name(),
                     "kernel_ms_per_launch": round(per_launch_ms, 4)},
        "conservation": {"sum_phi_rel_drift": (m1["sum_phi"] - m0["sum_phi"]) / m0["sum_phi"],
                         "sum_psi_rel_drift": (m1["sum_psi"] - m0["sum_psi"]) / m0["sum_psi"],
                         "steps": m1["step"]},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
