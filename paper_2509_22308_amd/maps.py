"""The paper's design maps through the batched engine, and the particle
trajectories they drive.

* run_map: the force/torque maps of arXiv 2509.22308 (Sec. IV.A,
  Fig. HS75_Map: metallo-dielectric, eps_r1 x phi0; Sec. IV.B, Fig. 2D_map:
  dielectric, eps_r2/eps_r1 x phi0 for eps_r1 = 1, 2, 5), every solve on the
  device through the engine (jlb_engine_*), reshaped to (rows, phi0).
* trajectory: the overdamped motion of Sec. IV.C through the library's
  jlb_trajectory (periodic cubic-spline interpolation of a map row in phi0,
  classical Runge-Kutta).

Command line (writes an .npz with the maps and a .json with the timings):

    python -m paper_2509_22308_amd.maps --map mdjc --out maps_mdjc
    python -m paper_2509_22308_amd.maps --map djc5 --stride 2 --out maps_djc5
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys
import time

import numpy as np

from . import _check, _vp, load
from .serve import run_design_map


def run_map(name: str, precision: str = "fp32", eps_stride: int = 1, phi_stride: int = 1, max_slots: int = 1024):
    import workloads
    if name == "mdjc":
        probs, rows, phi = workloads.paper_mdjc_map(eps_stride, phi_stride)
        row_key = "eps1"
    elif name.startswith("djc"):
        probs, rows, phi = workloads.paper_djc_map(float(name[3:]), eps_stride, phi_stride)
        row_key = "eps2_over_eps1"
    else:
        raise ValueError(f"unknown map {name!r} (mdjc, djc1, djc2, djc5)")
    out = run_design_map(probs, precision, max_slots=max_slots)
    res = out["results"]
    failed = [k for k, r in enumerate(res) if r["status"] != "done"]
    if failed:
        raise RuntimeError(f"{len(failed)} solves of map {name} did not finish (first: {failed[0]})")
    shape = (len(rows), len(phi))
    maps = {q: np.array([r[q] for r in res]).reshape(shape) for q in ("fx", "fy", "tz")}
    info = {"map": name, "precision": precision, "solves": len(probs), "rows": row_key,
            "wall_s": out["wall_s"], "lups": out["lups"], "solves_per_hour": out["solves_per_hour"],
            "peak_resident": out["peak_resident"], "nx": probs[0]["nx"], "radius": probs[0]["radius"],
            "wavelength": probs[0]["wavelength"], "steps": probs[0]["steps"]}
    return maps, np.array(rows), np.array(phi), info


def trajectory(phi_grid, fx, fy, tz, phi_start: float, t_end: float = 1e4, dt: float = 0.5,
               log_l_over_a: float = float(np.log(10.0)), record_every: int = 20):
    """Integrates Sec. IV.C's kinematics over a map row sampled at the uniform
    angles phi_grid (one period, without the repeated end point); returns
    arrays (t, x, y, phi) at every record_every-th step (phi unwrapped)."""
    phi_grid = np.asarray(phi_grid, dtype=np.float64)
    n = len(phi_grid)
    cols = [np.ascontiguousarray(v, dtype=np.float64) for v in (fx, fy, tz)]
    if any(len(c) != n for c in cols):
        raise ValueError("map rows and phi_grid differ in length")
    nsteps = int(round(t_end / dt))
    nrec = nsteps // record_every + 1
    out = np.zeros((nrec, 4))
    lib = load()
    _check(lib.jlb_trajectory(ctypes.c_int32(n), ctypes.c_double(phi_grid[0]), *[_vp(c.ctypes.data) for c in cols],
                              ctypes.c_double(phi_start), ctypes.c_double(dt), ctypes.c_int64(nsteps),
                              ctypes.c_double(log_l_over_a), ctypes.c_int32(record_every),
                              _vp(out.ctypes.data)))
    return out[:, 0], out[:, 1], out[:, 2], out[:, 3]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--map", required=True, help="mdjc, djc1, djc2 or djc5")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--stride", type=int, default=1, help="take every stride-th row and angle")
    ap.add_argument("--out", required=True, help="output path without extension")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    maps, rows, phi, info = run_map(args.map, args.precision, args.stride, args.stride)
    info["total_s"] = time.perf_counter() - t0
    np.savez_compressed(args.out + ".npz", rows=rows, phi=phi, **maps)
    with open(args.out + ".json", "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps(info), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
