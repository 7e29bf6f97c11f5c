"""Benchmark of the Janus-cylinder EM lattice Boltzmann hot path on one MI355X.

A "step" here is one complete solve of the hot path on synthetic input:
staircase geometry -> zeroed state -> 20000 fused stream-collide-boundary
lattice steps with the stress accumulation over the last 5 periods -> contour
reduction to F~x, F~y, M~z.  The workload is the dielectric Janus cylinder
eps1 = 2.25 / eps2 = 4.0, phi0 = 30 deg, a = 64, 1024 x 1024 grid,
lambda = 128, 20000 steps.  The value is lattice updates per second
(nx * ny * steps per solve / wall time per solve, conductor nodes included).

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def _kernel_of(precision: str) -> str:
    return {"fp64": "k_step_f64", "fp32": "k_step_neq<float>", "bf16": "k_step_neq<__bf16>"}[precision]


def gpu_leg(args):
    import torch

    import paper_2509_22308_amd as jlb
    import workloads

    torch.cuda.set_device(0)
    p = workloads.config2()
    prob = jlb.make_problem(p, args.precision)
    ws = torch.empty(jlb.jlb_workspace_size(prob), dtype=torch.uint8, device="cuda")
    lups_per_solve = p["nx"] * p["ny"] * p["steps"]

    for _ in range(args.warmup):
        jlb.jlb_solve(prob, ws)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(jlb.jlb_solve(prob, ws))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_per_solve = 1e3 * wall / args.steps
    value = lups_per_solve * args.steps / wall
    # dominant kernel: the fused step; HIP events on the library's stream
    # bracket the time loop of each solve (step kernels plus the small contour
    # kernels of the averaging window), so this is an upper bound on the
    # per-launch duration
    loop_ms = sum(r.loop_ms for r in results) / len(results)
    launch_ms = loop_ms / p["steps"]
    bytes_per_launch = results[0].bytes_per_step
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    r0 = results[0]

    extra = {"forces": {"fx": r0.fx, "fy": r0.fy, "tz": r0.tz},
             "loop_ms_per_solve": loop_ms, "graph_used": r0.graph_used,
             "bytes_per_lup": bytes_per_launch / (p["nx"] * p["ny"])}
    # the same step kernel, timed alone over back-to-back launches
    extra["step_kernel_ms_alone"] = jlb.jlb_time_step_kernel(prob, 20, 200, ws)
    if not args.quick:
        # a grid far larger than the 256 MB Infinity Cache: the HBM-bound figure
        big = workloads.problem(nx=4096, ny=4096, radius=256.0, kind="dielectric_janus", eps1=2.25, eps2=4.0,
                                phi0_deg=30.0, wavelength=512.0, steps=10000)
        for prec in ("fp64", "fp32", "bf16"):
            bp = jlb.make_problem(big, prec)
            bws = torch.empty(jlb.jlb_workspace_size(bp), dtype=torch.uint8, device="cuda")
            ms = jlb.jlb_time_step_kernel(bp, 5, 40, bws)
            per_lup = {"fp64": 177, "fp32": 89, "bf16": 57}[prec]
            gbs = 4096 * 4096 * per_lup / (ms * 1e-3) / 1e9
            extra[f"grid4096_{prec}"] = {"ms_per_step": ms, "glups": 4096 * 4096 / (ms * 1e-3) / 1e9,
                                        "gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
            del bws
        # the other precisions on the headline workload (one solve each)
        for prec in ("fp64", "fp32", "bf16"):
            if prec == args.precision:
                continue
            pp = jlb.make_problem(p, prec)
            pws = torch.empty(jlb.jlb_workspace_size(pp), dtype=torch.uint8, device="cuda")
            t = time.perf_counter()
            r = jlb.jlb_solve(pp, pws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            extra[f"config2_{prec}"] = {"glups": lups_per_solve / dt / 1e9, "ms_per_solve": 1e3 * dt,
                                        "loop_ms": r.loop_ms, "fx": r.fx, "fy": r.fy, "tz": r.tz}
            del pws
    roof = {"bound": "hbm", "kernel": _kernel_of(args.precision), "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": bytes_per_launch, "launch_ms": launch_ms}
    return p, value, ms_per_solve, roof, extra


def cpu_leg(p, budget_s: float = 15.0):
    """The FP64 oracle as it stands on the host cores, on a bounded sample:
    the headline workload's first n steps (n sized to about budget_s)."""
    from oracle import oracle

    threads = int(os.environ.get("JLB_ORACLE_THREADS", os.cpu_count() or 1))
    probe = dict(p, steps=20, avg_periods=0)
    t = time.perf_counter()
    oracle.solve(probe, fields=False, threads=threads)
    dt = time.perf_counter() - t
    n = max(20, min(p["steps"], int(20 * budget_s / max(dt, 1e-3))))
    sample = dict(p, steps=n, avg_periods=0)
    t = time.perf_counter()
    oracle.solve(sample, fields=False, threads=threads)
    dt = time.perf_counter() - t
    lups = p["nx"] * p["ny"] * n / dt
    return {"value": lups, "unit": "LUPS", "cores": threads, "kind": "oracle",
            "sample": f"{p['nx']}x{p['ny']} dielectric Janus, first {n} of {p['steps']} steps, "
                      f"reduced 11-population FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--quick", action="store_true", help="skip the extra precision and 4096^2 figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solves are independent and this build runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    p, value, ms, roof, extra = gpu_leg(args)
    cpu = None if args.no_cpu else cpu_leg(p)
    line = {
        "metric": "lattice updates/s and % HBM roofline; design-map solves/hour, p50/p99 latency",
        "value": value, "unit": "LUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16-storage/f32"}[args.precision],
        "data": "synthetic (parameter-defined scattering problem; no dataset)",
        "config": {"workload": "dielectric Janus cylinder eps 2.25/4.0, phi0 30 deg, a=64, 1024x1024, "
                               "lambda=128, 20000 steps, 5-period stress average (one full solve per step)",
                   "nx": p["nx"], "ny": p["ny"], "steps_per_solve": p["steps"], "precision": args.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
