"""Physics validation of the GPU path at the paper's working sizes.

Config 3 (metallo-dielectric Janus, a = 48 on a 768^2 grid, lambda = 96,
52 periods) against the analytic force and torque of Sec. IV.A (stored in
tests/golden/analytic_forces.json, written from oracle/analytic.py), the
symmetry law of Sec. IV.A.2, and the grid convergence of Sec. IV.A.2 at the
paper's point phi0 = 7 pi / 36, eps1 = 2, a / lambda = 1.
"""
import json
import math
import os

import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "analytic_forces.json")


@pytest.fixture(scope="module")
def jlb():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_22308_amd as J
    J.load()
    return J


def _golden(x, eps, deg):
    with open(GOLDEN) as f:
        g = json.load(f)["mdjc"]
    return [e for e in g if abs(e["x"] - x) < 1e-9 and abs(e["eps1"] - eps) < 1e-9 and abs(e["phi0_deg"] - deg) < 1e-9][0]


@pytest.mark.parametrize("eps1", [1.5, 2.0, 4.0, 8.0])
def test_config3_matches_papers_analytic_forces(jlb, eps1):
    """Sec. III quotes 5 % for lambda / dx >= 10 (here 96); lift and torque
    are held to 0.03 + 5 % of the value (they vanish on parts of the map)."""
    for deg in (0.0, 30.0, 90.0, 270.0):
        ref = _golden(math.pi, eps1, deg)
        p = W.config3(eps1, deg)
        print(f"[case] config3 eps1={eps1} phi0={deg}", flush=True)
        r = jlb.solve(p, "fp32")
        assert abs(r["fx"] - ref["fx"]) / ref["fx"] < 0.05, (eps1, deg, r["fx"], ref["fx"])
        for q in ("fy", "tz"):
            assert abs(r[q] - ref[q]) < 0.03 + 0.05 * abs(ref[q]), (eps1, deg, q, r[q], ref[q])


def test_config3_sweep_obeys_the_mirror_rule(jlb):
    for deg in (15.0, 45.0, 75.0):
        a = jlb.solve(W.config3(4.0, deg), "fp32")
        b = jlb.solve(W.config3(4.0, 180.0 - deg), "fp32")
        assert abs(a["fx"] - b["fx"]) < 1e-5 and abs(a["fy"] + b["fy"]) < 1e-5 and abs(a["tz"] + b["tz"]) < 1e-5


def test_grid_convergence_at_the_papers_point(jlb):
    """Sec. IV.A.2, Fig. (convergence): errors fall as a / dx grows (about
    second order in the paper, with fluctuations)."""
    ref = _golden(2 * math.pi, 2.0, math.degrees(7 * math.pi / 36))
    errs = []
    for a in (16, 32, 64):
        lam = float(a)  # a / lambda = 1
        p = W.problem(nx=8 * a, ny=8 * a, radius=float(a), kind="metallo_dielectric_janus", eps1=2.0,
                      phi0=7 * math.pi / 36, wavelength=lam, steps=W.steps_for(lam))
        r = jlb.solve(p, "fp64")
        e = max(abs(r[q] - ref[q]) / abs(ref[q]) for q in ("fx", "fy", "tz"))
        errs.append(e)
        print(f"[case] convergence a={a}: {r['fx']:.4f} {r['fy']:.4f} {r['tz']:.4f} max rel err {e:.4f}", flush=True)
    assert errs[-1] < errs[0]
    assert errs[-1] < 0.05
