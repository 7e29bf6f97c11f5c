"""Summarise the paper's design maps computed on the GPU (results/maps_*.npz,
written by ``python -m paper_2509_22308_amd.maps``) and the trajectories they
drive, into results/design_maps.md.

Compared with: the values the paper prints (tests/golden/paper_values.json)
and, for the metallo-dielectric map, the analytic solution on a subgrid
(tests/golden/mdjc_map_analytic.json).  Trajectories (Sec. IV.C) come from
the library's jlb_trajectory over map rows at the paper's parameters.
Run from the repository root:

    python results/make_summary.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from scipy.interpolate import CubicSpline  # noqa: E402

from paper_2509_22308_amd.maps import trajectory  # noqa: E402

RES = os.path.join(ROOT, "results")


def load(name):
    d = np.load(os.path.join(RES, f"maps_{name}.npz"))
    with open(os.path.join(RES, f"maps_{name}.json")) as f:
        info = json.load(f)
    return {k: d[k] for k in d.files}, info


def at(m, rows, phi, row, ang):
    i = int(np.argmin(np.abs(rows - row)))
    j = int(np.argmin(np.abs(phi - ang)))
    return {q: float(m[q][i, j]) for q in ("fx", "fy", "tz")}, rows[i], phi[j]


def trajectories(m, rows, phi, row, lines, label):
    i = int(np.argmin(np.abs(rows - row)))
    fx, fy, tz = m["fx"][i, :-1], m["fy"][i, :-1], m["tz"][i, :-1]
    for p0 in (0.0, math.pi / 4, 7 * math.pi / 6):
        t, x, y, p = trajectory(phi[:-1], fx, fy, tz, p0, t_end=1e4, dt=0.5)
        end = p[-1] % (2 * math.pi)
        # the torque there, on the same periodic cubic spline the integrator uses
        per = CubicSpline(np.append(phi[:-1], phi[0] + 2 * math.pi), np.append(tz, tz[0]), bc_type="periodic")
        m_end = float(per(phi[0] + (end - phi[0]) % (2 * math.pi)))
        lines.append(f"| {label} | {rows[i]:.2f} | {p0 / math.pi:.3f} π | {end / math.pi:.3f} π | "
                     f"{x[-1]:.0f} | {y[-1]:.0f} | {m_end:.1e} |")


def main():
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        pv = json.load(f)
    lines = ["# Design maps and trajectories (arXiv 2509.22308, Sec. IV)", "",
             "Written by `results/make_summary.py` from the maps in `results/maps_*.npz` "
             "(FP32, every solve through the batched engine on one MI355X).", ""]
    lines += ["## Runs", "", "| map | solves | grid | a | λ | steps | wall s | solves/h | GLUPS |", "|---|---|---|---|---|---|---|---|---|"]
    maps = {}
    for name in ("mdjc", "djc1", "djc2", "djc5"):
        try:
            maps[name] = load(name)
        except FileNotFoundError:
            continue
        d, info = maps[name]
        lines.append(f"| {name} | {info['solves']} | {info['nx']}² | {info['radius']:.0f} | {info['wavelength']:.0f} | "
                     f"{info['steps']} | {info['wall_s']:.1f} | {info['solves_per_hour']:.0f} | {info['lups'] / 1e9:.1f} |")
    lines.append("")
    if "mdjc" in maps:
        d, _ = maps["mdjc"]
        rows, phi = d["rows"], d["phi"]
        r = pv["mdjc_ranges"]
        lines += ["## Metallo-dielectric map (Sec. IV.A, Fig. HS75_Map)", "",
                  "| quantity | this map | paper (printed) |", "|---|---|---|",
                  f"| F̃x range | {d['fx'].min():.3f} … {d['fx'].max():.3f} | {r['fx_min']} … {r['fx_max']} |",
                  f"| max \\|F̃y\\| | {np.abs(d['fy']).max():.3f} | ≈ {r['fy_absmax']} |",
                  f"| max \\|M̃z\\| | {np.abs(d['tz']).max():.3f} | ≈ {r['tz_absmax']} |"]
        for pt in pv["mdjc_points"]:
            v, e, f = at(d, rows, phi, pt["eps1"], pt["phi0_over_pi"] * math.pi)
            lines.append(f"| F̃x at ε_r1 = {e:.2f}, φ0 = {f / math.pi:.3f} π ({pt['what']}) | {v['fx']:.3f} | ≈ {pt['fx']} |")
        with open(os.path.join(ROOT, "tests", "golden", "mdjc_map_analytic.json")) as f:
            g = json.load(f)
        ge, gp = np.array(g["eps1"]), np.array(g["phi0"])
        errs = {q: [] for q in ("fx", "fy", "tz")}
        for a, e in enumerate(ge):
            i = int(np.argmin(np.abs(rows - e)))
            for b, p in enumerate(gp):
                j = int(np.argmin(np.abs(phi - p)))
                for q in errs:
                    ref = g[q][a][b]
                    errs[q].append(abs(d[q][i, j] - ref) / (abs(ref) if q == "fx" else 1.0))
        dr = np.array(errs["fx"])
        lines += ["", f"Against the analytic solution on {len(dr)} points (every other row and angle; "
                      "Fig. HS75_Map (d)–(f) shows the paper's own error map):", "",
                  "| | median | 95th pct | max |", "|---|---|---|---|",
                  f"| drag, relative | {np.median(dr):.4f} | {np.percentile(dr, 95):.4f} | {dr.max():.4f} |",
                  f"| lift, absolute | {np.median(errs['fy']):.4f} | {np.percentile(errs['fy'], 95):.4f} | {max(errs['fy']):.4f} |",
                  f"| torque, absolute | {np.median(errs['tz']):.4f} | {np.percentile(errs['tz'], 95):.4f} | {max(errs['tz']):.4f} |",
                  ""]
    djc = [n for n in ("djc1", "djc2", "djc5") if n in maps]
    if djc:
        rr = pv["djc_ranges"]
        lines += ["## Dielectric maps (Sec. IV.B, Fig. 2D_map)", "",
                  "| ε_r1 | F̃x range | paper | max \\|F̃y\\| | max \\|M̃z\\| |", "|---|---|---|---|---|"]
        for n in djc:
            d, _ = maps[n]
            e1 = n[3:]
            pr = rr.get(f"eps1_{e1}", {})
            lines.append(f"| {e1} | {d['fx'].min():.3f} … {d['fx'].max():.3f} | {pr.get('fx_min')} … {pr.get('fx_max')} | "
                         f"{np.abs(d['fy']).max():.3f} | {np.abs(d['tz']).max():.3f} |")
        lines += ["", f"Paper: peak lift {rr['fy_absmax_range'][0]}–{rr['fy_absmax_range'][1]}, "
                      f"peak torque {rr['tz_absmax_range'][0]}–{rr['tz_absmax_range'][1]} across the three.", ""]
        if "djc5" in maps:
            d, _ = maps["djc5"]
            rows, phi = d["rows"], d["phi"]
            i = int(np.argmin(np.abs(rows - 4.0)))
            row = d["fx"][i, :91]
            lines += [f"ε_r1 = 5, ε_r2/ε_r1 = 4 over φ0 ∈ [0, π]: drag min {row.min():.3f} at "
                      f"{phi[int(np.argmin(row))] / math.pi:.3f} π, max {row.max():.3f} at "
                      f"{phi[int(np.argmax(row))] / math.pi:.3f} π (paper: ≈ 0.8 at π/180, ≈ 1.73 at 11π/30).", ""]
            j = int(np.argmin(np.abs(phi - math.pi / 2)))
            sl = [(rows[k], d["fx"][k, j]) for k in range(len(rows)) if 3.4 <= rows[k] <= 3.9]
            lines += ["ε_r1 = 5, φ0 = π/2, drag along ε_r2/ε_r1 (paper: valley at 3.60, peak at 3.66): " +
                      ", ".join(f"{a:.2f}: {b:.3f}" for a, b in sl), ""]
    lines += ["## Trajectories (Sec. IV.C)", "",
              "log(l/a) = log 10 (the paper does not state l/a; positions scale with it, the orientation does not); "
              "t̃ up to 10 000, RK4 step 0.5, periodic cubic spline over the map row in φ0.", "",
              "| map | row (ε_r1 or ε_r2/ε_r1) | φ0(0) | φ0(t̃_f) mod 2π | x̃(t̃_f) | ỹ(t̃_f) | M̃z at the end |",
              "|---|---|---|---|---|---|---|"]
    if "mdjc" in maps:
        d, _ = maps["mdjc"]
        for e in (1.0, 2.0, 5.0):
            trajectories(d, d["rows"], d["phi"], e, lines, "MDJC")
    for n in djc:
        d, _ = maps[n]
        trajectories(d, d["rows"], d["phi"], 2.0, lines, f"DJC ε_r1 = {n[3:]}")
    lines.append("")
    with open(os.path.join(RES, "design_maps.md"), "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
