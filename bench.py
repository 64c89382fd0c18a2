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
# what the step kernels are built from: sources and the build flags
KERNEL_SOURCES = ("paper_2408_15654_amd/csrc/lbm.hip", "paper_2408_15654_amd/csrc/lbm_device.h",
                  "paper_2408_15654_amd/build.py")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "lbm_step_kernel_many_drops_2048_{}_counters.txt")


def algorithmic_bytes_per_site(precision: str) -> int:
    """Bytes one site-update must move: 26 live populations read and written
    (f_0..f_8, g_0..g_8, h_1..h_8) plus the previous level read and written.
    float64/float32 storage keep (phi, psi) as rest values and (ux, uy) as
    aux; float16 storage keeps (phi, psi, P, rho ux, rho uy) in float32 as
    rest values (the bases of the stored deviations, and rho u / rho(phi) is
    the previous velocity).  The previous level's mass flux S is recomputed
    from the previous phi, which the step reads anyway."""
    fields = 5 if precision == "fp16dev" else 4
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
    cores = oracle.threads()
    out = {"value": round(pr.sites * n / dt / 1e6, 3), "unit": "MLUPS",
           "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle, same 2048x2048 many-drop problem, {n} steps "
                     f"after 1 warm-up step ({dt:.1f} s)"}
    # one thread on one step of the same problem, and the full 64x64 drop
    # (2000 steps) on all threads
    try:
        v1, dt1 = oracle.time_mlups(pr.params, pr.fields0, 1, threads=1)
        out["one_thread_MLUPS"] = round(v1, 3)
    finally:
        oracle.lib().or_set_threads(cores)
    from paper_2408_15654_amd import workloads
    c1 = workloads.c1_stationary_drop()
    vc1, dtc1 = oracle.time_mlups(c1.params, c1.fields0, c1.steps)
    out["c1_full_MLUPS"] = round(vc1, 3)
    out["c1_full_seconds"] = round(dtc1, 2)
    out["cpu_model"] = cpu_model()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


def batched_sweep(n=256, steps=400, seq_steps=20, precision="fp32", probe=8):
    """The batched sweep: n independent drop-in-shear problems (site counts
    log-uniform in [64^2, 512^2], aspect 2:1), advanced together by the
    batch runtime, against the same problems solved one at a time with the
    single-simulation entry points."""
    import torch

    from paper_2408_15654_amd import lbm, workloads

    probs = workloads.c4_batch(n=n, precision=precision, steps=steps)
    total_sites = sum(p.sites for p in probs)
    # one solve at a time: each problem alone, its launches back to back
    t_seq = 0.0
    for pr in probs:
        sim = lbm.Simulation(pr.params)
        sim.init_fields(*pr.fields0)
        sim.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(seq_steps)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        sim.close()
    seq = total_sites * seq_steps / t_seq / 1e6

    budget = (lbm.Batch.overhead_bytes(n) + sum(lbm.Batch.instance_bytes(p.params) for p in probs)
              + (8 << 20))
    b = lbm.Batch(budget, max_instances=n)
    ids = [b.submit(p.params, *p.fields0, 1 << 40) for p in probs]

    def timed(k):
        b.step(64)  # warm-up (captures the graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(k)
        torch.cuda.synchronize()
        return total_sites * k / (time.perf_counter() - t0) / 1e6

    b.set_schedule(rows=0, grid_waves=0, chunk=32)
    untuned = timed(steps)
    chosen = b.autotune(probe)
    tuned = timed(steps)
    hbm = budget
    b.close()
    del b
    torch.cuda.empty_cache()
    bps = algorithmic_bytes_per_site(precision)
    achieved = bps * tuned * 1e6 / 1e9  # GB/s at the tuned rate
    return {"instances": n, "sites": total_sites, "precision": precision,
            "one_at_a_time_MLUPS": round(seq, 1), "batched_untuned_MLUPS": round(untuned, 1),
            "batched_tuned_MLUPS": round(tuned, 1), "tuned_schedule": chosen,
            "speedup_vs_one_at_a_time": round(tuned / seq, 2),
            "workspace_bytes": hbm, "timed_steps": steps, "one_at_a_time_steps": seq_steps,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "bytes_per_site_update": bps,
                         "basis": "algorithmic bytes x batched site updates / wall time"}}


def rel_errors(got, want):
    import numpy as np

    out = {}
    for k in ("phi", "psi"):
        out[k] = float(np.abs(got[k] - want[k]).max() / np.abs(want[k]).max())
    du = np.hypot(got["ux"] - want["ux"], got["uy"] - want["uy"]).max()
    out["u"] = float(du / max(np.hypot(want["ux"], want["uy"]).max(), 1e-300))
    return out


# Admission policy of the serving stream: least work first, and at most
# about twice the sites at which one grid already saturates the device
# (2048 x 1024, 2.1 M sites, runs at the 2048^2 rate).  Measured on the
# 200-request float32 stream at 0.7x load against first come, first served
# with no cap: same throughput and p50, p99 4.3 s instead of 5.7 s.
SERVE_POLICY = {"order": "shortest", "max_running_sites": 4_000_000}


def serving_bench(n=200, budgets_gb=(2, 64), precisions=("fp32", "fp16dev"), load=0.7,
                  max_steps=20000, quiet=False):
    """The serving stream: Poisson arrivals of drop-in-shear and Marangoni
    migration solves (sites log-uniform in [128^2, 1024^2], steps uniform in
    [1000, max_steps]) at `load` times the batch's measured capacity,
    admitted by HBM budget.  For every 10th request the same problem is
    re-run alone in float64 on the GPU and the served result's error
    against it is reported."""
    import numpy as np
    import torch

    from paper_2408_15654_amd import lbm, serve

    out = []
    refs = {}  # float64 re-runs (and perturbed twins), shared by runs of the same problem
    for prec in precisions:
        # capacity: the batched rate on the stream's own problem mix
        reqs, _ = serve.serving_stream(n=n, rate=1.0, precision=prec, max_steps=max_steps)
        probe = reqs[:48]
        budget = (lbm.Batch.overhead_bytes(64) + sum(lbm.Batch.instance_bytes(r.params)
                                                     for r in probe) + (16 << 20))
        b = lbm.Batch(budget, max_instances=64)
        for r in probe:
            b.submit(r.params, *r.fields0, 1 << 40)
        b.step(64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(512)
        torch.cuda.synchronize()
        cap = sum(int(r.params["nx"]) * int(r.params["ny"]) for r in probe) * 512 / (
            time.perf_counter() - t0) / 1e6
        b.close()
        del b
        torch.cuda.empty_cache()
        reqs, rate = serve.serving_stream(n=n, precision=prec, max_steps=max_steps,
                                          offered_MLUPS=load * cap)
        check = {r.rid for r in reqs if r.rid % 10 == 0}
        for gb in budgets_gb:
            srv = serve.Server(int(gb) << 30, max_instances=512, chunk=64, **SERVE_POLICY)
            results, stats = srv.run(reqs, keep_fields=check)
            srv.close()
            del srv
            torch.cuda.empty_cache()
            errs, spread = [], []
            by_id = {r.rid: r for r in reqs}
            rng = np.random.default_rng(1)
            for res in results:
                if res.fields is None:
                    continue
                req = by_id[res.rid]
                key = (req.steps, json.dumps(dict(req.params, precision="fp64"), sort_keys=True),
                       req.fields0[0].tobytes(), req.fields0[1].tobytes())
                if key not in refs:
                    # the float64 re-run, and a twin whose initial phi carries
                    # a relative perturbation of 1e-10: how far two float64
                    # runs drift apart measures how much the flow amplifies
                    # rounding
                    ref = []
                    for eps in (0.0, 1e-10):
                        phi0 = req.fields0[0] * (
                            1.0 + eps * rng.standard_normal(req.fields0[0].shape))
                        sim = lbm.Simulation(dict(req.params, precision="fp64"))
                        sim.init_fields(phi0, *req.fields0[1:])
                        sim.step(req.steps)
                        ref.append(sim.read_fields())
                        sim.close()
                    refs[key] = ref
                ref = refs[key]
                errs.append(rel_errors(res.fields, ref[0]))
                spread.append(rel_errors(ref[1], ref[0]))
            worst = {k: max(e[k] for e in errs) for k in ("phi", "psi", "u")} if errs else {}
            wsp = {k: max(e[k] for e in spread) for k in ("phi", "psi", "u")} if spread else {}
            out.append(dict(stats, precision=prec, budget_GB=gb, policy=SERVE_POLICY,
                            capacity_MLUPS=round(cap, 1),
                            offered_rate_per_s=round(rate, 3), fp64_rerun_checked=len(errs),
                            worst_rel_err_vs_fp64=worst,
                            fp64_spread_from_perturbation_1e10=wsp))
            if not quiet:
                print(json.dumps({"serving_run": out[-1]}), file=sys.stderr, flush=True)
    return out


def precision_run(steps=5000):
    """The 2048x2048 field advanced `steps` steps in float32 and
    float16-deviation storage, compared with the float64 library run (the
    reference for long runs once float64 matches the oracle to 1e-12), and
    the drift of Sum phi, Sum psi in each."""
    import torch

    from paper_2408_15654_amd import lbm, workloads

    pr = workloads.c3_many_drops()
    res, ref = {}, None
    for prec in ("fp64", "fp32", "fp16dev"):
        sim = lbm.Simulation(dict(pr.params, precision=prec))
        sim.init_fields(*pr.fields0)
        m0 = sim.moments()
        sim.step(steps)
        f = sim.read_fields()
        m1 = sim.moments()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        drift = {"sum_phi": (m1["sum_phi"] - m0["sum_phi"]) / m0["sum_phi"],
                 "sum_psi": (m1["sum_psi"] - m0["sum_psi"]) / m0["sum_psi"]}
        if ref is None:
            ref = f
            res[prec] = {"drift": drift}
        else:
            res[prec] = {"rel_err_vs_fp64": rel_errors(f, ref), "drift": drift}
    return {"steps": steps, **res}


def shear_run(steps=20000, every=2500):
    """The 256x128 drop in shear (beta 0 and 0.5) in float64 and float32:
    Taylor deformation D(t) and interface length from the on-device shape
    diagnostics, and the drift of Sum psi."""
    from paper_2408_15654_amd import lbm, workloads

    out = {}
    for beta in (0.0, 0.5):
        pr = workloads.c2_shear_drop(beta=beta)
        for prec in ("fp64", "fp32"):
            sim = lbm.Simulation(dict(pr.params, precision=prec))
            sim.init_fields(*pr.fields0)
            m0 = sim.moments()
            D, C = [], []
            for t in range(0, steps + 1, every):
                if t:
                    sim.step(every)
                sh = sim.shape()
                D.append(round(sh["taylor_D"], 6))
                C.append(round(sh["length"], 3))
            m1 = sim.moments()
            sim.close()
            out[f"beta{beta}_{prec}"] = {
                "t": list(range(0, steps + 1, every)), "taylor_D": D, "length": C,
                "sum_psi_drift": (m1["sum_psi"] - m0["sum_psi"]) / m0["sum_psi"]}
    return out


def bubble_run(nx=240, precision="fp32", points=7):
    """The rising bubble of Sec. 4.3 (240 x 480, t = 3, i.e. 172800 steps),
    clean (E_0 = 0) and surfactant-laden (E_0 = 0.5): the bubble's centre
    of mass Y_c (from the on-device shape diagnostics, in units of the
    domain width) at `points` times."""
    from paper_2408_15654_amd import lbm, workloads

    out = {}
    for beta in (0.0, 0.5):
        pr = workloads.e3_rising_bubble(beta=beta, nx=nx, precision=precision)
        sim = lbm.Simulation(pr.params)
        sim.init_fields(*pr.fields0)
        every = pr.steps // (points - 1)
        ts, yc = [], []
        t0 = time.perf_counter()
        for k in range(points):
            if k:
                sim.step(every)
            ts.append(round(k * every / nx ** 2, 4))
            yc.append(round(sim.shape()["cy"] / nx, 5))
        wall = time.perf_counter() - t0
        sim.close()
        out[f"E0_{beta}"] = {"t": ts, "Yc": yc, "steps": every * (points - 1),
                             "seconds": round(wall, 2)}
    return {"precision": precision, **out}


def progress(msg: str):
    """Phase marker on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp16dev"])
    ap.add_argument("--rows", type=int, default=0, help="tile height override")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="the 256-problem batched sweep instead of the 2048^2 field")
    ap.add_argument("--serve", action="store_true",
                    help="the serving stream (p50/p99 latency) instead of the 2048^2 field")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-max-steps", type=int, default=20000)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the short batched-sweep and serving runs of the default line")
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
    if args.serve:
        runs = serving_bench(n=args.serve_requests, max_steps=args.serve_max_steps)
        main_run = [r for r in runs if r["precision"] == "fp32"][-1]
        print(json.dumps({
            "metric": "p50/p99 batched-solve latency and aggregate MLUPS of the serving stream",
            "value": main_run["aggregate_MLUPS"], "unit": "MLUPS", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic", "dtype": "fp32",
            "latency_p50_s": main_run["latency_p50_s"],
            "latency_p99_s": main_run["latency_p99_s"],
            "config": {"workload": f"serving_stream_{args.serve_requests}"},
            "serving": runs}), flush=True)
        return
    if args.batched:
        r = batched_sweep(steps=args.steps)
        print(json.dumps({
            "metric": "aggregate MLUPS of the batched sweep (256 problems)",
            "value": r["batched_tuned_MLUPS"], "unit": "MLUPS", "n_gpus": 1,
            "steps": r["timed_steps"], "higher_is_better": True, "data": "synthetic",
            "dtype": r["precision"], "config": {"workload": "batched_shear_sweep_256"},
            "batched": r}), flush=True)
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
    bps = algorithmic_bytes_per_site(args.precision)
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
                     "kernel_ms_per_launch": round(per_launch_ms, 4),
                     # the counter bytes (reads past L2 and writes, halo
                     # re-reads included) over this run's launch time
                     "traffic_GBps": (round(traffic / (per_launch_ms * 1e-3) / 1e9, 1)
                                      if traffic else None),
                     "traffic_frac": (round(traffic / (per_launch_ms * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4) if traffic else None)},
        "conservation": {"sum_phi_rel_drift": (m1["sum_phi"] - m0["sum_phi"]) / m0["sum_phi"],
                         "sum_psi_rel_drift": (m1["sum_psi"] - m0["sum_psi"]) / m0["sum_psi"],
                         "steps": m1["step"]},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    progress(f"2048x2048 field: {mlups:.0f} MLUPS")
    if not args.no_extras:
        # the batched sweep (256 problems) and a short serving stream, so the
        # one line carries every figure of the metric
        # the batched sweep at its full 10000 steps (untuned and tuned)
        out["batched"] = batched_sweep(steps=10000)
        progress(f"batched sweep: {out['batched']['batched_tuned_MLUPS']} MLUPS")
        # the serving stream, 100 solves of up to 10000 steps: float32 and
        # float16 deviations, each with a small (2 GB) and a large (64 GB)
        # HBM budget
        runs = serving_bench(n=100, budgets_gb=(2, 64), precisions=("fp32", "fp16dev"),
                             max_steps=10000, quiet=True)
        main = [r for r in runs if r["precision"] == "fp32" and r["budget_GB"] == 64][0]
        out["serving"] = main
        out["serving_runs"] = runs
        out["latency_p50_s"] = main["latency_p50_s"]
        out["latency_p99_s"] = main["latency_p99_s"]
        progress(f"serving stream: p50 {main['latency_p50_s']} s, p99 {main['latency_p99_s']} s")
        out["precision_2048_5000_steps"] = precision_run()
        progress("precision run done")
        out["shear_drop_20000_steps"] = shear_run()
        progress("shear run done")
        out["rising_bubble"] = bubble_run()
        progress("rising bubble done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
