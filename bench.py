"""Benchmark of the Janus-cylinder EM lattice Boltzmann hot path on one MI355X.

Default (the contract line): a "step" is one complete solve of the hot path
on synthetic input -- staircase geometry -> zeroed state -> 20000 fused
stream-collide-boundary lattice steps with the stress accumulation over the
last 5 periods -> contour reduction to F~x, F~y, M~z -- for the dielectric
Janus cylinder eps1 = 2.25 / eps2 = 4.0, phi0 = 30 deg, a = 64 on a
1024 x 1024 grid, lambda = 128.  value = lattice updates per second
(nx * ny * steps per solve / wall time per solve, conductor nodes included).
The same line carries, in extra, the rest of the metric measured on the same
GPU: config 4's design map (solves/hour, against one-at-a-time FP64 solves)
and config 5's serving run on the first 64 of its seeded arrivals (p50 / p99
latency, throughput).  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]

Other modes (one JSON line each):
    --workload designmap [--fraction f]   config 4: 576 dielectric Janus solves
                                          (a ~ U{32..128}) batched by the engine,
                                          vs one-at-a-time FP64 solves
    --workload serve [--requests n]       config 5: Poisson arrivals (20/s),
                                          byte-budget admission, p50/p99 latency
    --kernel-only                         the fused step kernel and the copy
                                          reference alone (for rocprofv3 passes)
    --summarize DIR --out FILE            turn rocprofv3 CSV output into a
                                          short text summary under profiles/
    --record-traffic / --record-valu KEY  merge FETCH_SIZE / WRITE_SIZE or VALU
                                          counter passes into profiles/*.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# FP32 vector issue peak for this arithmetic: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz, one FP32 add or multiply per lane per cycle.  The update uses
# neither packed FP32 (left out of every build) nor FMA contraction (off, so
# that every kernel variant rounds the same operations the same way), so the
# 157.3 TFLOP/s of packed FMA is out of its reach.
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# FP32 / BF16 deviation update, interior node: three rest populations (5 each),
# four outgoing pairs (3 each), the three moments (4 + 1, 4 + 1, 4 + 1) and the
# eight new deviations (2 x 4 + 4): adds, subtracts and multiplies
FLOPS_PER_LUP = {"fp32": 54, "bf16": 54}
BYTES_PER_LUP = {"fp64": 177, "fp32": 89, "bf16": 57}
KERNEL_NAME = {"fp64": "k_step_f64", "fp32": "k_step_neq*<float>", "bf16": "k_step_neq*<__bf16>"}
TWO_STEP_KERNEL_NAME = {"fp64": "k_step2_f64", "fp32": "k_step2_neq<float>", "bf16": "k_step2_neq<__bf16>"}
MULTI_STEP_KERNEL_NAME = {"fp32": "k_stepm_neq<float>", "bf16": "k_stepm_neq<__bf16>"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "step_valu.json")
DEVICE_SRCS = [os.path.join(ROOT, "paper_2509_22308_amd", "csrc", n)
               for n in ("jlb_device.hip", "jlb_device_f64.hip", "jlb_device_common.h", "jlb_internal.h")]


def kernel_source_hash() -> str:
    """Hash of every source the device code is built from: counters recorded
    for another hash describe other kernels and are not used."""
    h = hashlib.sha256()
    for path in DEVICE_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _workspace(jlb, prob):
    import torch
    return torch.empty(jlb.jlb_workspace_size(prob), dtype=torch.uint8, device="cuda")


def measured_traffic(precision: str, variant: int):
    """Bytes per launch of the step kernel leaving L2 (to the Infinity Cache
    and HBM), from the committed counter summary, or None when it was taken
    on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    e = t.get("config2", {}).get(precision, {}).get(str(variant))
    return e.get("l2_egress_bytes_per_launch") if e else None


def measured_valu(precision: str, variant: int):
    """VALU counters per launch of the step kernel from the committed summary
    (VALUBusy, VALU instructions, waves), or None when they were taken on a
    different kernel source."""
    try:
        with open(VALU_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("config2", {}).get(precision, {}).get(str(variant))


def _chosen_kernels(jlb, prob, ws, prec: str, launches: int):
    """Autotune, then time the chosen kernels: ms per launch of the best
    single step and (FP32 / BF16, when the autotuner selected them) of the
    two-step and multi-step kernels."""
    best, tune = jlb.jlb_autotune(prob, launches, ws)
    one = jlb.jlb_time_step_kernel(prob, 5, 4 * launches, ws)
    two = multi = None
    if jlb.jlb_get_two_step_variant(jlb.PRECISIONS[prec]) >= 0:
        two = jlb.jlb_time_two_step_kernel(prob, 5, 2 * launches, ws)
    if prec != "fp64" and jlb.jlb_get_multi_step_variant(jlb.PRECISIONS[prec]) >= 0:
        multi = jlb.jlb_time_multi_step_kernel(prob, 5, launches, ws)
    return best, tune, one, two, multi


def gpu_leg(args):
    import torch

    import paper_2509_22308_amd as jlb
    import workloads

    torch.cuda.set_device(0)
    p = workloads.config2()
    prob = jlb.make_problem(p, args.precision)
    ws = _workspace(jlb, prob)
    # the autotuner picks the step kernels (tile shape; single, two- or multi-step)
    # for this device and grid
    variant, tune_ms = jlb.jlb_autotune(prob, 20, ws)
    two_variant = jlb.jlb_get_two_step_variant(jlb.PRECISIONS[args.precision])
    multi_variant = jlb.jlb_get_multi_step_variant(jlb.PRECISIONS[args.precision]) if args.precision != "fp64" else -1
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
    # Dominant kernel: the one that runs the whole periods before the
    # averaging window (most of the solve), replayed from a hipGraph.  The
    # library brackets that stretch with HIP events on its stream, so
    # main_ms / main_launches is that kernel's mean launch duration over the
    # timed solves.  A launch advances the state by `depth` lattice steps,
    # i.e. depth x nx x ny lattice updates at the algorithmic bytes per update.
    loop_ms = sum(r.loop_ms for r in results) / len(results)
    r0 = results[0]
    passes = r0.state_passes
    main_kind, main_variant = r0.main_kind, r0.main_variant
    depth = {1: 1, 2: 2}.get(main_kind) or jlb.jlb_multi_step_shape(main_variant)[0]
    launch_ms = sum(r.main_ms for r in results) / sum(r.main_launches for r in results)
    bytes_per_pass = r0.bytes_per_step
    extra = {"forces": {"fx": r0.fx, "fy": r0.fy, "tz": r0.tz}, "loop_ms_per_solve": loop_ms,
             "state_passes_per_solve": passes, "graph_used": r0.graph_used,
             "main_stretch": {"kind": {1: "single step", 2: "two-step", 3: "multi-step"}[main_kind],
                              "ms_per_solve": r0.main_ms, "launches_per_solve": r0.main_launches},
             "step_variant": jlb.STEP_VARIANTS.get(jlb.jlb_get_step_variant(jlb.PRECISIONS[args.precision]))
             if args.precision != "fp64" else jlb.FP64_STEP_VARIANTS.get(variant),
             "two_step_variant": (jlb.FP64_TWO_STEP_VARIANTS if args.precision == "fp64" else jlb.TWO_STEP_VARIANTS
                                  ).get(two_variant) if two_variant >= 0 else None,
             "multi_step_variant": jlb.MULTI_STEP_VARIANTS.get(multi_variant) if multi_variant >= 0 else None,
             "autotune_ms_per_step": [round(m, 5) for m in tune_ms],
             "step_kernel_ms_alone": jlb.jlb_time_step_kernel(prob, 20, 200, ws)}
    if two_variant >= 0:
        extra["two_step_kernel_ms_alone"] = jlb.jlb_time_two_step_kernel(prob, 10, 100, ws)
    if multi_variant >= 0:
        extra["multi_step_kernel_ms_alone"] = jlb.jlb_time_multi_step_kernel(prob, 10, 100, ws)
    if not args.quick:
        nb = 4 << 30
        ms = jlb.jlb_copy_bandwidth(nb, 10)
        extra["copy_4GiB_GBps"] = 2 * nb / (ms * 1e-3) / 1e9
        # a grid far larger than the 256 MB Infinity Cache: the HBM-bound figure
        big = workloads.problem(nx=4096, ny=4096, radius=256.0, kind="dielectric_janus", eps1=2.25, eps2=4.0,
                                phi0_deg=30.0, wavelength=512.0, steps=10000)
        nodes = 4096 * 4096
        for prec in ("fp64", "fp32", "bf16"):
            bp = jlb.make_problem(big, prec)
            bws = _workspace(jlb, bp)
            best, _, one, two, multi = _chosen_kernels(jlb, bp, bws, prec, 10)
            gbs = nodes * BYTES_PER_LUP[prec] / (one * 1e-3) / 1e9
            ent = {"single_step": {"variant": (jlb.FP64_STEP_VARIANTS if prec == "fp64" else jlb.STEP_VARIANTS).get(
                       jlb.jlb_get_step_variant(jlb.PRECISIONS[prec])), "ms_per_launch": one,
                       "glups": nodes / (one * 1e-3) / 1e9, "gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}}
            if two is not None:
                gbs2 = nodes * BYTES_PER_LUP[prec] / (two * 1e-3) / 1e9
                names = jlb.FP64_TWO_STEP_VARIANTS if prec == "fp64" else jlb.TWO_STEP_VARIANTS
                ent["two_step"] = {"variant": names.get(jlb.jlb_get_two_step_variant(jlb.PRECISIONS[prec])),
                                   "ms_per_launch": two, "glups": 2 * nodes / (two * 1e-3) / 1e9,
                                   "gbs": gbs2, "hbm_frac": gbs2 / HBM_PEAK_GBS}
            if multi is not None:
                mv = jlb.jlb_get_multi_step_variant(jlb.PRECISIONS[prec])
                depth, _ = jlb.jlb_multi_step_shape(mv)
                gbsm = nodes * BYTES_PER_LUP[prec] / (multi * 1e-3) / 1e9
                ent["multi_step"] = {"variant": jlb.MULTI_STEP_VARIANTS.get(mv), "ms_per_launch": multi,
                                     "glups": depth * nodes / (multi * 1e-3) / 1e9, "gbs": gbsm,
                                     "hbm_frac": gbsm / HBM_PEAK_GBS}
            extra[f"grid4096_{prec}"] = ent
            del bws
        for prec in ("fp64", "fp32", "bf16"):
            if prec == args.precision:
                continue
            pp = jlb.make_problem(p, prec)
            pws = _workspace(jlb, pp)
            jlb.jlb_autotune(pp, 10, pws)
            t = time.perf_counter()
            r = jlb.jlb_solve(pp, pws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            extra[f"config2_{prec}"] = {"glups": lups_per_solve / dt / 1e9, "ms_per_solve": 1e3 * dt,
                                        "loop_ms": r.loop_ms, "fx": r.fx, "fy": r.fy, "tz": r.tz}
            del pws
    if main_kind == 3:
        kname = f"{MULTI_STEP_KERNEL_NAME[args.precision]} ({jlb.MULTI_STEP_VARIANTS.get(main_variant)})"
        index = len(jlb.STEP_VARIANTS) + len(jlb.TWO_STEP_VARIANTS) + main_variant
    elif main_kind == 2:
        names = jlb.FP64_TWO_STEP_VARIANTS if args.precision == "fp64" else jlb.TWO_STEP_VARIANTS
        kname = f"{TWO_STEP_KERNEL_NAME[args.precision]} ({names.get(main_variant)})"
        index = len(jlb.STEP_VARIANTS) + main_variant
    else:
        kname = KERNEL_NAME[args.precision]
        index = main_variant
    roof = roofline(args.precision, kname, index, depth, bytes_per_pass, p["nx"] * p["ny"], launch_ms,
                    r0.main_launches)
    return p, value, ms_per_solve, roof, extra


def roofline(precision, kname, index, depth, bytes_per_pass, nodes, launch_ms, launches_per_solve):
    """Roofline of the dominant kernel against the resource that bounds it.

    A launch advances the state by `depth` lattice steps; it must read and
    write the state once (bytes_per_pass), and it performs depth x nodes
    lattice updates of FLOPS_PER_LUP operations each.  The VALU counter pass
    of profiles/step_valu.json (VALUBusy: the share of the launch's cycles
    the SIMDs spend issuing vector ALU instructions) decides the bound: at
    0.6 or more the launch is bound by VALU issue and is placed against the
    FP32 issue peak with its algorithmic operations; otherwise against the
    HBM peak with one state pass per launch."""
    secs = launch_ms * 1e-3
    per_pass_gbs = bytes_per_pass / secs / 1e9
    flops = FLOPS_PER_LUP.get(precision, 0) * depth * nodes
    tflops = flops / secs / 1e12
    valu = measured_valu(precision, index)
    traffic = measured_traffic(precision, index)
    valu_bound = valu is not None and valu.get("valu_busy", 0.0) >= 0.6 and flops > 0
    if valu_bound:
        head = {"bound": "alu", "achieved": tflops, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / VALU_FP32_PEAK_TFLOPS}
    else:
        head = {"bound": "hbm", "achieved": per_pass_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": per_pass_gbs / HBM_PEAK_GBS}
    head.update({
        "traffic": traffic, "kernel": kname, "steps_per_launch": depth, "launch_ms": launch_ms,
        "launches_per_solve": launches_per_solve,
        "algorithmic_flops_per_launch": flops, "flops_per_update": FLOPS_PER_LUP.get(precision),
        "per_pass": {"bytes": bytes_per_pass, "gbs": per_pass_gbs, "frac_of_hbm": per_pass_gbs / HBM_PEAK_GBS},
        "equiv_gbs": depth * bytes_per_pass / secs / 1e9,
        "counters": valu,
        "note": ("bound from the VALUBusy counter of the same kernel source (profiles/step_valu.json). achieved = "
                 f"{FLOPS_PER_LUP.get(precision)} FP32 operations per lattice update x {depth} x nx x ny updates per "
                 "launch / mean launch duration (HIP events around the graph-replayed periods before the window), "
                 f"peak = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = {VALU_FP32_PEAK_TFLOPS:.1f} TFLOP/s (no packed "
                 "FP32, no FMA contraction). per_pass: one read and one write of the state per launch against 8 "
                 "TB/s. equiv_gbs: the algorithmic bytes of every update the launch performs (temporal blocking "
                 "moves them once per launch). traffic: FETCH_SIZE + WRITE_SIZE per launch, scaled by a copy "
                 "kernel of known size: bytes leaving L2, Infinity-Cache hits included (not DRAM bytes).")
                if valu_bound else
                ("achieved = one read and one write of the state per launch / mean launch duration against 8 TB/s; "
                 "traffic: FETCH_SIZE + WRITE_SIZE per launch scaled by a copy kernel (bytes leaving L2)."),
    })
    return head
    return p, value, ms_per_solve, roof, extra


def cpu_leg(p, budget_s: float = 15.0, threads: int = 0):
    """The FP64 oracle as it stands, on the host cores (all of them, or
    `threads`), on a bounded sample: the headline workload's first n steps
    (n sized to about budget_s)."""
    from oracle import oracle

    threads = threads or int(os.environ.get("JLB_ORACLE_THREADS", os.cpu_count() or 1))
    probe = dict(p, steps=20, avg_periods=0)
    t = time.perf_counter()
    oracle.solve(probe, fields=False, threads=threads)
    dt = time.perf_counter() - t
    n = max(20, min(p["steps"], int(20 * budget_s / max(dt, 1e-3))))
    sample = dict(p, steps=n, avg_periods=0)
    t = time.perf_counter()
    oracle.solve(sample, fields=False, threads=threads)
    dt = time.perf_counter() - t
    return {"value": p["nx"] * p["ny"] * n / dt, "unit": "LUPS", "cores": threads, "kind": "oracle",
            "sample": f"{p['nx']}x{p['ny']} dielectric Janus, first {n} of {p['steps']} steps, "
                      f"reduced 11-population FP64, {dt:.1f} s"}


def base_line(args, metric_value, ms, config, roof=None, cpu=None, extra=None, dtype=None):
    return {
        "metric": "lattice updates/s and % HBM roofline; design-map solves/hour, p50/p99 latency",
        "value": metric_value, "unit": "LUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype or {"fp64": "f64", "fp32": "f32", "bf16": "bf16-storage/f32"}[args.precision],
        "data": "synthetic (parameter-defined scattering problems; no dataset)",
        "config": config, "roofline": roof, "cpu_baseline": cpu, "extra": extra or {},
    }


def run_default(args):
    p, value, ms, roof, extra = gpu_leg(args)
    if not args.quick:
        # the rest of the metric, on the same GPU: design-map solves/hour
        # (config 4, all 576 solves) and serving p50 / p99 (config 5, the
        # first 64 arrivals of its seeded sequence)
        print("[bench] design map (config 4)", file=sys.stderr, flush=True)
        extra["design_map"] = design_map_leg(args.precision)
        print("[bench] serving (config 5, 64 requests)", file=sys.stderr, flush=True)
        extra["serving"] = serve_leg(args.precision, 64, 16, 256, 256, "fifo")
    cpu = None if args.no_cpu else cpu_leg(p)
    if cpu is not None:
        # the same oracle on one host thread, a shorter sample
        extra["cpu_baseline_single_thread"] = cpu_leg(p, budget_s=6.0, threads=1)
    config = {"workload": "dielectric Janus cylinder eps 2.25/4.0, phi0 30 deg, a=64, 1024x1024, lambda=128, "
                          "20000 steps, 5-period stress average (one full solve per step)",
              "nx": p["nx"], "ny": p["ny"], "steps_per_solve": p["steps"], "precision": args.precision}
    return base_line(args, value, ms, config, roof, cpu, extra)


def _kernel_choice(jlb, prec: str, four_step=None) -> dict:
    """The step kernels the autotuner left selected for prec, and the engine's
    four-step shape as it timed it on the resident mix (four_step: the
    engine's report)."""
    if prec == "fp64":
        return {"single_step": jlb.FP64_STEP_VARIANTS.get(jlb.jlb_get_step_variant(0))}
    p = jlb.PRECISIONS[prec]
    two, multi = jlb.jlb_get_two_step_variant(p), jlb.jlb_get_multi_step_variant(p)
    shape = four_step["variant"] if four_step and four_step.get("variant") else None
    return {"single_step": jlb.STEP_VARIANTS.get(jlb.jlb_get_step_variant(p)),
            "two_step": jlb.TWO_STEP_VARIANTS.get(two) if two >= 0 else None,
            "multi_step": jlb.MULTI_STEP_VARIANTS.get(multi) if multi >= 0 else None,
            "engine_rounds": (f"{shape}, two-step for each solve's last one to three steps" if two >= 0 and shape
                              else "two-step" if two >= 0 else "single steps"),
            "engine_four_step_timing": four_step}


def design_map_leg(precision: str, fraction: float = 1.0):
    """Config 4: the design map through the engine, and the one-at-a-time
    plain FP64 baseline on the same GPU (a sample stratified by radius,
    extrapolated by lattice-update count)."""
    import torch

    import paper_2509_22308_amd as jlb
    import workloads
    from paper_2509_22308_amd.serve import run_design_map

    probs = workloads.config4_sweep()
    if fraction < 1.0:
        probs = probs[:: max(1, int(round(1.0 / fraction)))]
    jlb.jlb_autotune(jlb.make_problem(probs[0], precision), 10)
    out = run_design_map(probs, precision)
    # baseline: one-at-a-time plain FP64 solves on the same GPU, timed on a
    # seeded sample stratified by radius, extrapolated by LUP count
    order = sorted(range(len(probs)), key=lambda k: probs[k]["radius"])
    sample = [probs[order[int(q * (len(order) - 1))]] for q in (0.0, 0.33, 0.66, 1.0)]
    t = time.perf_counter()
    for sp in sample:
        jlb.solve(sp, "fp64")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    lups_sample = sum(sp["nx"] * sp["ny"] * sp["steps"] for sp in sample)
    base_lups = lups_sample / dt
    total = sum(pp["nx"] * pp["ny"] * pp["steps"] for pp in probs)
    extra = {"solves": len(probs), "wall_s": out["wall_s"], "solves_per_hour": out["solves_per_hour"],
             "peak_resident": out["peak_resident"],
             "baseline_fp64_one_at_a_time": {"lups": base_lups, "solves_per_hour_extrapolated":
                                             len(probs) / (total / base_lups) * 3600.0,
                                             "sample": "4 solves stratified by radius"},
             "failed": sum(1 for r in out["results"] if r["status"] != "done"),
             "kernels": _kernel_choice(jlb, precision, out.get("four_step")), "lups": out["lups"],
             "precision": precision,
             "workload": f"config 4 design map: {len(probs)} dielectric Janus solves, eps2/eps1 1.1..10 "
                         f"(16 log-spaced) x 36 orientations, a ~ U{{32..128}}, grid 8a, lambda 2a, 52 periods"}
    return extra


def run_designmap(args):
    import torch
    torch.cuda.set_device(0)
    extra = design_map_leg(args.precision, args.fraction)
    config = {"workload": extra["workload"], "precision": args.precision}
    return base_line(args, extra["lups"], 1e3 * extra["wall_s"], config, extra=extra)


def serve_leg(precision: str, requests: int, a_min: int, a_max: int, slots: int, policy: str):
    """Config 5: seeded Poisson arrivals served by the engine (continuous
    batching, byte-budget admission); latency from arrival to completion."""
    import paper_2509_22308_amd as jlb
    import workloads
    from paper_2509_22308_amd.serve import serve

    reqs = workloads.config5_requests(n_req=requests, a_min=a_min, a_max=a_max)
    jlb.jlb_autotune(jlb.make_problem(reqs[0][1], precision), 10)
    out = serve(reqs, precision, max_slots=slots, policy=policy)
    extra = {k: out[k] for k in ("requests", "completed", "wall_s", "p50_s", "p99_s", "mean_s", "queue_p50_s",
                                 "queue_p99_s", "submit_delay_p50_s", "submit_delay_p99_s", "solves_per_hour",
                                 "throughput_lups", "offered_lups", "peak_resident", "budget_bytes", "policy",
                                 "max_slots")}
    extra["kernels"] = _kernel_choice(jlb, precision, out.get("four_step"))
    extra["precision"] = precision
    extra["workload"] = (f"config 5 serving: the first {requests} of the seeded Poisson arrivals at 20/s "
                         f"(seed 22308), dielectric Janus a ~ U{{{a_min}..{a_max}}}, grid 8a, eps ~ U[1.5,10], "
                         "lambda 2a, 52 periods, byte-budget admission")
    return extra


def run_serve(args):
    import torch
    torch.cuda.set_device(0)
    extra = serve_leg(args.precision, args.requests, args.a_min, args.a_max, args.slots, args.policy)
    config = {"workload": extra["workload"], "precision": args.precision}
    return base_line(args, extra["throughput_lups"], 1e3 * extra["wall_s"], config, extra=extra)


def run_kernel_only(args):
    """The fused step kernel of the headline workload and the copy reference,
    alone: the command the rocprofv3 counter passes profile."""
    import torch

    import paper_2509_22308_amd as jlb
    import workloads

    torch.cuda.set_device(0)
    if args.grid:
        n = args.grid
        p = workloads.problem(nx=n, ny=n, radius=n / 16, kind="dielectric_janus", eps1=2.25, eps2=4.0,
                              phi0_deg=30.0, wavelength=n / 8, steps=10000)
    else:
        p = workloads.config2()
    prob = jlb.make_problem(p, args.precision)
    ws = _workspace(jlb, prob)
    if args.multi_step >= 0:
        jlb.jlb_set_multi_step_variant(jlb.PRECISIONS[args.precision], args.multi_step)
        variant = len(jlb.STEP_VARIANTS) + len(jlb.TWO_STEP_VARIANTS) + args.multi_step
        ms = jlb.jlb_time_multi_step_kernel(prob, 2, args.launches, ws)
    elif args.two_step >= 0:
        # the two-step kernel alone (counter passes serialise kernels, which
        # would mislead the autotuner: the variant is given)
        jlb.jlb_set_two_step_variant(jlb.PRECISIONS[args.precision], args.two_step)
        variant = len(jlb.STEP_VARIANTS) + args.two_step
        ms = jlb.jlb_time_two_step_kernel(prob, 2, args.launches, ws)
    else:
        if args.variant >= 0:
            jlb.jlb_set_step_variant(jlb.PRECISIONS[args.precision], args.variant)
            variant = args.variant
        else:
            variant, _ = jlb.jlb_autotune(prob, 5, ws)
            variant = jlb.jlb_get_step_variant(jlb.PRECISIONS[args.precision])
        ms = jlb.jlb_time_step_kernel(prob, 2, args.launches, ws)
    copy_bytes = 1 << 30
    cms = jlb.jlb_copy_bandwidth(copy_bytes, 3)
    print(json.dumps({"mode": "kernel-only", "grid": [p["nx"], p["ny"]], "precision": args.precision, "variant": variant,
                      "step_ms": ms, "launches": args.launches, "bytes_per_launch": BYTES_PER_LUP[args.precision]
                      * p["nx"] * p["ny"], "copy_bytes": copy_bytes, "copy_ms": cms,
                      "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def summarize(args):
    """Short text summary of rocprofv3 CSV output (kernel stats or counters)."""
    lines = [f"# rocprofv3 summary ({os.path.basename(os.path.normpath(args.summarize))})",
             f"command: {args.command}" if args.command else "", ""]
    stats = glob.glob(os.path.join(args.summarize, "**", "*kernel_stats.csv"), recursive=True)
    for path in stats:
        with open(path) as f:
            rows = list(csv.DictReader(f))
        lines.append("## kernel stats (" + os.path.basename(path) + ")")
        lines.append("| kernel | calls | total ms | average us | percent |")
        lines.append("|---|---|---|---|---|")
        for r in rows[:15]:
            name = r.get("Name", "")[:90]
            lines.append(f"| {name} | {r.get('Calls')} | {float(r.get('TotalDurationNs', 0)) / 1e6:.3f} | "
                         f"{float(r.get('AverageNs', 0)) / 1e3:.3f} | {float(r.get('Percentage', 0)):.2f} |")
        lines.append("")
    ctrs = glob.glob(os.path.join(args.summarize, "**", "*counter_collection.csv"), recursive=True)
    for path in ctrs:
        agg = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (r.get("Kernel_Name", "")[:90], r.get("Counter_Name", ""))
                agg.setdefault(key, []).append(float(r.get("Counter_Value", 0.0)))
        lines.append("## counters per dispatch (" + os.path.basename(path) + ")")
        lines.append("| kernel | counter | dispatches | mean | min | max |")
        lines.append("|---|---|---|---|---|---|")
        for (k, c), v in sorted(agg.items()):
            lines.append(f"| {k} | {c} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
        lines.append("")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(args.out)


def _counter_means(d: str, counter: str) -> dict:
    """Mean value of one counter per kernel name over a rocprofv3 CSV output folder."""
    agg = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    agg.setdefault(r.get("Kernel_Name", ""), []).append(float(r.get("Counter_Value", 0.0)))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def record_traffic(args):
    """Bytes per launch of the step kernel leaving L2, from a FETCH_SIZE and a
    WRITE_SIZE pass of --kernel-only, each scaled so that the plain copy
    kernel of the same run reads its known byte count, merged into the
    traffic file under (workload, precision, variant)."""
    fetch = _counter_means(args.fetch_dir, "FETCH_SIZE")
    write = _counter_means(args.write_dir, "WRITE_SIZE")
    copy_bytes = float(1 << 30)  # --kernel-only copies 1 GiB

    def pick(table, copy):
        step = [v for k, v in table.items() if "k_step" in k]
        cp = [v for k, v in table.items() if "k_copy" in k]
        if len(step) != 1 or len(cp) != 1:
            raise SystemExit(f"expected one step and one copy kernel, found {list(table)}")
        return step[0], copy / (cp[0] * 1024.0)

    f_kib, f_scale = pick(fetch, copy_bytes)
    w_kib, w_scale = pick(write, copy_bytes)
    entry = {"variant": args.variant, "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
             "fetch_scale": f_scale, "write_scale": w_scale,
             "l2_egress_bytes_per_launch": f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale, "command": args.command}
    try:
        with open(args.out) as f:
            t = json.load(f)
    except OSError:
        t = {}
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        t = {}
    t["kernel_source_sha256_16"] = kernel_source_hash()
    t.setdefault(args.record_traffic, {}).setdefault(args.precision, {})[str(args.variant)] = entry
    with open(args.out, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    print(json.dumps(entry))


def record_valu(args):
    """VALU counters per launch of the step kernel from one rocprofv3 --pmc
    pass of --kernel-only (VALUBusy, SQ_INSTS_VALU, SQ_WAVES,
    GRBM_GUI_ACTIVE), merged into the VALU file under (workload, precision,
    variant) with the kernel source hash."""
    vals = {c: _counter_means(args.valu_dir, c) for c in ("VALUBusy", "SQ_INSTS_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE")}

    def step(table):
        v = [x for k, x in table.items() if "k_step" in k]
        if len(v) != 1:
            raise SystemExit(f"expected one step kernel, found {list(table)}")
        return v[0]

    busy = step(vals["VALUBusy"])
    insts, waves = step(vals["SQ_INSTS_VALU"]), step(vals["SQ_WAVES"])
    entry = {"variant": args.variant, "valu_busy": busy / 100.0, "valu_insts_per_launch": insts,
             "waves_per_launch": waves, "valu_insts_per_wave": insts / waves if waves else None,
             "gui_active_cycles": step(vals["GRBM_GUI_ACTIVE"]), "command": args.command}
    try:
        with open(args.out) as f:
            t = json.load(f)
    except OSError:
        t = {}
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        t = {}
    t["kernel_source_sha256_16"] = kernel_source_hash()
    t.setdefault(args.record_valu, {}).setdefault(args.precision, {})[str(args.variant)] = entry
    with open(args.out, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    print(json.dumps(entry))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--workload", default="config2", choices=["config2", "designmap", "serve"])
    ap.add_argument("--fraction", type=float, default=1.0, help="designmap: take every (1/f)-th solve")
    ap.add_argument("--requests", type=int, default=64, help="serve: number of requests")
    ap.add_argument("--a-min", type=int, default=16)
    ap.add_argument("--a-max", type=int, default=64)
    ap.add_argument("--policy", default="fifo", choices=["fifo", "sjf"], help="serve: engine admission order")
    ap.add_argument("--slots", type=int, default=256, help="serve: most solves resident at once")
    ap.add_argument("--quick", action="store_true",
                    help="skip the extra precision, 4096^2, copy, design-map and serving figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--kernel-only", action="store_true")
    ap.add_argument("--launches", type=int, default=50)
    ap.add_argument("--grid", type=int, default=0, help="kernel-only: an n x n grid instead of config 2")
    ap.add_argument("--variant", type=int, default=-1, help="kernel-only: this step variant instead of the autotuner's")
    ap.add_argument("--two-step", type=int, default=-1, help="kernel-only: time this two-step variant instead")
    ap.add_argument("--multi-step", type=int, default=-1, help="kernel-only: time this multi-step variant instead")
    ap.add_argument("--summarize", default=None)
    ap.add_argument("--record-traffic", default=None, help="workload key (config2, grid4096): merge counter passes")
    ap.add_argument("--record-valu", default=None, help="workload key (config2): merge a VALU counter pass")
    ap.add_argument("--valu-dir", default=None)
    ap.add_argument("--fetch-dir", default=None)
    ap.add_argument("--write-dir", default=None)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.record_traffic:
        record_traffic(args)
        return
    if args.record_valu:
        record_valu(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs each solve on a single MI355X (independent solves "
              "shard across GPUs with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.kernel_only:
        run_kernel_only(args)
        return
    line = {"config2": run_default, "designmap": run_designmap, "serve": run_serve}[args.workload](args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
