"""Design-map sweeps and a request loop on top of the batched engine.

Both drive the C ABI's engine (jlb_engine_*): every lattice step, boundary,
stress average and reduction runs in the library's kernels; this module only
submits problems, advances the engine and collects results and timings.

* run_design_map: a sweep of independent solves (the force/torque design
  diagrams of arXiv 2509.22308, Sec. IV.A / IV.B, are such sweeps), all
  submitted at once and batched by the engine.
* serve: requests arriving at given times (Poisson arrivals in the
  benchmark), submitted when they arrive while earlier ones run; reports
  latency from arrival to completion (p50/p99) next to throughput.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import Engine, make_problem, jlb_workspace_size


def _engine_budget(problems, precision, budget_bytes):
    if budget_bytes is not None:
        return int(budget_bytes)
    import torch
    free, _ = torch.cuda.mem_get_info()
    need = sum(jlb_workspace_size(make_problem(p, precision)) for p in problems)
    return int(min(0.8 * free, 1.05 * need + (64 << 20)))


def run_design_map(problems, precision: str = "fp32", budget_bytes: int | None = None, max_slots: int = 1024,
                   steps_per_call: int = 1024) -> dict:
    """Solve every problem through the engine; returns results and timings."""
    budget = _engine_budget(problems, precision, budget_bytes)
    eng = Engine(budget, max_slots)
    t0 = time.perf_counter()
    tickets = [eng.submit(make_problem(p, precision)) for p in problems]
    peak = 0
    last = t0
    while True:
        eng.run(steps_per_call)
        st = eng.stats()
        peak = max(peak, st["resident"])
        if st["queued"] == 0 and st["resident"] == 0:
            break
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            print(f"[design map] {st['finished']}/{len(problems)} done, {st['resident']} resident, "
                  f"{last - t0:.0f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    results = []
    for t in tickets:
        status, res = eng.poll(t)
        results.append(dict(res.as_dict(), status=status))
    four = eng.four_step_choice(precision) if precision != "fp64" else None
    eng.close()
    lups = float(sum(p["nx"] * p["ny"] * p["steps"] for p in problems))
    return {"results": results, "wall_s": wall, "lups": lups / wall, "solves_per_hour": len(problems) / wall * 3600.0,
            "peak_resident": peak, "budget_bytes": budget, "four_step": four}


def serve(requests, precision: str = "fp32", budget_bytes: int | None = None, max_slots: int = 256,
          steps_per_call: int = 128, time_scale: float = 1.0, policy: str = "fifo") -> dict:
    """Replay (arrival_seconds, problem) requests in wall-clock time.

    Requests are submitted when their arrival time has passed; the engine
    admits them as memory and slots free up (in arrival order, or smallest
    work first with policy "sjf") and steps every resident solve together.
    Latency = completion time - arrival time; queue wait = admission time -
    submission time (the engine's clocks); submission delay = submission
    time - arrival time (the host loop submits between engine calls, each
    one captured chunk of steps_per_call steps by default).
    """
    reqs = sorted(requests, key=lambda r: r[0])
    budget = _engine_budget([p for _, p in reqs], precision, budget_bytes)
    eng = Engine(budget, max_slots)
    eng.set_policy(policy)
    outstanding = {}
    done = []
    k = 0
    peak = 0
    t0 = time.perf_counter()
    last = t0
    while k < len(reqs) or outstanding:
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            print(f"[serve] {len(done)}/{len(reqs)} done, {len(outstanding)} outstanding, {last - t0:.0f} s",
                  file=sys.stderr, flush=True)
        now = time.perf_counter() - t0
        while k < len(reqs) and reqs[k][0] * time_scale <= now:
            t = eng.submit(make_problem(reqs[k][1], precision))
            # arrival -> submission: the time the request waited for the
            # host loop, which is inside eng.run while earlier work runs
            outstanding[t] = (k, reqs[k][0] * time_scale, time.perf_counter() - t0)
            k += 1
        st = eng.stats()
        if st["resident"] == 0 and st["queued"] == 0:
            if k < len(reqs):
                time.sleep(max(0.0, min(0.01, reqs[k][0] * time_scale - (time.perf_counter() - t0))))
            continue
        eng.run(steps_per_call)
        peak = max(peak, eng.stats()["resident"])
        now = time.perf_counter() - t0
        for t in list(outstanding):
            status, res = eng.poll(t)
            if status in ("done", "failed", "cancelled"):
                idx, arr, sub = outstanding.pop(t)
                # the engine's own clocks: submit -> done (total_ms), admit -> done (loop_ms)
                done.append({"index": idx, "status": status, "arrival_s": arr, "done_s": now,
                             "latency_s": now - arr, "queue_s": max(0.0, (res.total_ms - res.loop_ms) * 1e-3),
                             "submit_delay_s": sub - arr, "fx": res.fx, "fy": res.fy, "tz": res.tz})
    wall = time.perf_counter() - t0
    four = eng.four_step_choice(precision) if precision != "fp64" else None
    eng.close()
    lat = np.array([d["latency_s"] for d in done if d["status"] == "done"])
    wait = np.array([d["queue_s"] for d in done if d["status"] == "done"])
    sub = np.array([d["submit_delay_s"] for d in done if d["status"] == "done"])
    lups = float(sum(p["nx"] * p["ny"] * p["steps"] for _, p in reqs))
    span = reqs[-1][0] * time_scale if reqs else 0.0
    return {
        "requests": len(reqs), "completed": int(len(lat)), "wall_s": wall,
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_s": float(lat.mean()) if len(lat) else None,
        "queue_p50_s": float(np.percentile(wait, 50)) if len(wait) else None,
        "queue_p99_s": float(np.percentile(wait, 99)) if len(wait) else None,
        "submit_delay_p50_s": float(np.percentile(sub, 50)) if len(sub) else None,
        "submit_delay_p99_s": float(np.percentile(sub, 99)) if len(sub) else None,
        "policy": policy, "max_slots": max_slots,
        "throughput_lups": lups / wall, "solves_per_hour": len(lat) / wall * 3600.0,
        "offered_lups": lups / span if span > 0 else None, "peak_resident": peak, "budget_bytes": budget,
        "four_step": four, "done": sorted(done, key=lambda d: d["index"]),
    }
