"""Pins of the analytic validator (oracle/analytic.py) on the CPU.

The closed forms of Sec. IV.A are held to a direct quadrature of the stress
integrals of Sec. II.B and to an independent far-field momentum balance; the
metallo-dielectric solution is held to the values the paper prints and to
its symmetry laws.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special

from oracle import analytic as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


def _golden():
    with open(os.path.join(GOLDEN, "analytic_forces.json")) as f:
        return json.load(f)


def test_bessel_ratio_recurrences_match_scipy_where_scipy_is_finite():
    for z in (1.3, math.pi, 7.9):
        M = 40
        m = np.arange(M + 1)
        hr, inv = A._hankel_ratios(z, M)
        h = special.hankel1(m, z)
        assert np.allclose(hr, special.h1vp(m, z) / h, rtol=1e-10)
        assert np.allclose(inv, 1.0 / h, rtol=1e-10)
        jr = A._bessel_j_ratio(z, M)
        assert np.allclose(jr, special.jvp(m, z) / special.jv(m, z), rtol=1e-8)


@pytest.mark.parametrize("kind", ["mie", "pec", "mdjc"])
def test_closed_forms_equal_stress_quadrature_and_far_field_balance(kind):
    x, phi0 = math.pi, 0.7
    if kind == "mie":
        c = A.mie_coeffs(x, 3.0, phi0)
    elif kind == "pec":
        c = A.pec_coeffs(x, phi0)
    else:
        c = A.mdjc_coeffs(x, 2.5, phi0, 257)
    fx, fy, tz = A.forces_closed_form(*c, x, phi0)
    qx, qy, qt = A.forces_quadrature(*c, x, phi0)
    ffx, ffy = A.forces_far_field(*c, x, phi0)
    # Eqs. (U), (V), (Torque) vs Eqs. (drag), (lift), (Torque) integrated directly
    assert abs(fx - qx) < 1e-10 and abs(fy - qy) < 1e-10 and abs(tz - qt) < 1e-10
    # momentum balance from the scattered far field alone (lossless: extinction = scattering)
    assert abs(fx - ffx) < 1e-9 and abs(fy - ffy) < 1e-9
    if kind != "mdjc":
        assert abs(fy) < 1e-12 and abs(tz) < 1e-12


def test_textbook_cylinder_limits():
    # the drag efficiency of a perfectly reflecting cylinder falls monotonically
    # between a/lambda = 0.25, 0.5 and 1 and stays above the specular value
    vals = [A.forces_closed_form(*A.pec_coeffs(2 * math.pi * r), 2 * math.pi * r, 0.0)[0] for r in (0.25, 0.5, 1.0)]
    assert vals[0] > vals[1] > vals[2] > 1.5
    # a vanishing contrast scatters nothing
    x = math.pi
    assert abs(A.forces_closed_form(*A.mie_coeffs(x, 1.0 + 1e-12), x, 0.0)[0]) < 1e-9


def test_papers_printed_drag_values_at_a_over_lambda_one():
    g = {(round(e["eps1"], 2), round(e["phi0_deg"], 6)): e for e in _golden()["mdjc"]
         if abs(e["a_over_lambda"] - 1.0) < 1e-12}
    for pt in _paper()["mdjc_points"]:
        key = (round(pt["eps1"], 2), round(math.degrees(pt["phi0_over_pi"] * math.pi), 6))
        ref = g[key]
        # printed values carry about two significant digits and are LBM values (Sec. IV.A.2)
        assert abs(ref["fx"] - pt["fx"]) < 0.02 * pt["fx"] + 0.01, (pt, ref["fx"])


def test_printed_extrema_are_extrema_of_the_analytic_solution():
    x = 2 * math.pi
    N = 257
    f = lambda e, p: A.mdjc_forces(x, e, p, N)[0]  # noqa: E731
    # App. B Case 1: local minimum of drag along phi0 at eps1 = 2, phi0 = 7 pi / 90
    p0 = 7 * math.pi / 90
    d = math.pi / 90
    assert f(2.0, p0) < f(2.0, p0 - 2 * d) and f(2.0, p0) < f(2.0, p0 + 2 * d)
    # App. B Case 2: drag peak near eps1 = 3.56 and valley near 4 at phi0 = pi / 2
    assert f(3.56, math.pi / 2) > f(3.4, math.pi / 2) and f(3.56, math.pi / 2) > f(3.72, math.pi / 2)
    assert f(4.0, math.pi / 2) < f(3.84, math.pi / 2) and f(4.0, math.pi / 2) < f(4.16, math.pi / 2)


def test_analytic_symmetry_about_half_pi():
    x, N = math.pi, 257
    for eps in (1.5, 4.0):
        for deg in (10.0, 35.0, 200.0):
            p = math.radians(deg)
            a = A.mdjc_forces(x, eps, p, N)
            b = A.mdjc_forces(x, eps, math.pi - p, N)
            assert abs(a[0] - b[0]) < 1e-9 and abs(a[1] + b[1]) < 1e-9 and abs(a[2] + b[2]) < 1e-9
        for p in (math.pi / 2, 1.5 * math.pi):
            q = A.mdjc_forces(x, eps, p, N)
            assert abs(q[1]) < 1e-9 and abs(q[2]) < 1e-9


def test_pec_facing_drag_approaches_pec_cylinder():
    # Sec. IV.A.2 / App. A: phi0 = 3 pi / 2 resembles a homogeneous PEC cylinder
    x = 2 * math.pi
    pec = A.forces_closed_form(*A.pec_coeffs(x), x, 0.0)[0]
    g = [e for e in _golden()["mdjc"] if abs(e["a_over_lambda"] - 1.0) < 1e-12 and e["phi0_deg"] == 270.0][0]
    assert abs(g["fx"] - pec) / pec < 0.03


def test_richardson_extrapolation_is_consistent_with_the_finest_solve():
    for e in _golden()["mdjc"]:
        assert abs(e["fx"] - e["fx_N4097"]) < 5e-4 * max(1.0, abs(e["fx"]))
        assert 1.0 < e["order"] < 1.6 or abs(e["fx"] - e["fx_N4097"]) < 1e-6
