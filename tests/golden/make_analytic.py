"""Write the stored analytic force/torque values used by the oracle tests.

Calls only oracle/analytic.py (arXiv 2509.22308 Sec. IV.A: Eqs. integral
equation, constants_Bm_Dm, coefficients, U, V, Torque; Sec. II: Mie and PEC
series follow from Eqs. incident field and scattered field with full-circle
boundary conditions).  Run from the repository root:

    python tests/golden/make_analytic.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import analytic as A  # noqa: E402


def main():
    out = {"note": "analytic (F~x, F~y, M~z); MDJC values Richardson-extrapolated over N, 2N-1, 4N-3 "
                   "with M = N - 1 modes; written by tests/golden/make_analytic.py",
           "mdjc": [], "mie": [], "pec": []}
    cases = []
    x_half = math.pi  # a / lambda = 0.5
    for eps in (1.5, 2.0, 4.0, 8.0):
        for deg in (0.0, 30.0, 90.0, 270.0):
            cases.append((x_half, eps, deg))
    x_one = 2 * math.pi  # a / lambda = 1, the paper's size
    for eps, phi in ((2.0, 7 * math.pi / 36), (2.0, 7 * math.pi / 90), (2.0, math.pi / 2),
                     (3.56, math.pi / 2), (4.0, math.pi / 2), (2.0, 3 * math.pi / 2)):
        cases.append((x_one, eps, math.degrees(phi)))
    for x, eps, deg in cases:
        q, p, raw = A.mdjc_forces_extrapolated(x, eps, math.radians(deg), N=1025)
        out["mdjc"].append({"x": x, "a_over_lambda": x / (2 * math.pi), "eps1": eps, "phi0_deg": deg,
                            "fx": q[0], "fy": q[1], "tz": q[2], "order": p,
                            "fx_N4097": float(raw[2][0])})
        print(out["mdjc"][-1], flush=True)
    for x, eps in ((math.pi / 2, 2.0), (math.pi, 2.25), (math.pi, 4.0), (math.pi, 10.0), (math.pi, 2.0),
                   (2 * math.pi, 2.0)):
        c = A.mie_coeffs(x, eps, 0.0)
        out["mie"].append({"x": x, "eps": eps, "fx": A.forces_closed_form(*c, x, 0.0)[0]})
    for aol in (0.25, 0.5, 1.0):
        x = 2 * math.pi * aol
        c = A.pec_coeffs(x, 0.0)
        out["pec"].append({"x": x, "a_over_lambda": aol, "fx": A.forces_closed_form(*c, x, 0.0)[0]})
    with open(os.path.join(ROOT, "tests", "golden", "analytic_forces.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
