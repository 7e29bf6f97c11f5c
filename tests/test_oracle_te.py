"""Pins of the oracle's TE^z polarisation (Hz, Ex, Ey), the case arXiv
2509.22308 leaves for later work (Sec. I), on the same lattice and printed
equations (Sec. III).  All run on the CPU.

* The reduced 11-population TE^z form equals the literal 42-scalar printed
  update (which evolves the TE^z components once the source excites them).
* Vacuum duality: without a body, TE^z (Hz, Ex, Ey) equals TM^z (Ez, -Hx, -Hy).
* Symmetry laws and the exact conserved norm hold as in TM^z.
* Whole solves against textbook TE^z series: a dielectric cylinder (Mie) and a
  conducting cylinder, forces and far field.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import analytic as A
from oracle import oracle as O


def _te(p):
    return dict(p, polarization="te")


@pytest.mark.parametrize("kind", ["homogeneous", "dielectric_janus", "metallo_dielectric_janus"])
def test_literal_and_reduced_te_forms_agree(kind):
    p = _te(W.problem(nx=72, ny=66, radius=12.0, kind=kind, eps1=3.0, eps2=6.5, phi0_deg=37.0, wavelength=24.0,
                      steps=900, avg_periods=2))
    a = O.solve(p, literal=False)
    b = O.solve(p, literal=True)
    scale = max(np.max(np.abs(a["ez"])), np.max(np.abs(a["hy"])))
    assert scale > 0.1
    for f in ("ez", "hx", "hy"):
        assert np.max(np.abs(a[f] - b[f])) <= 1e-13 * scale
    for q in ("fx", "fy", "tz"):
        assert abs(a[q] - b[q]) <= 1e-12 * max(1.0, abs(a[q]))


def test_vacuum_duality_with_tm():
    """No body (radius below one cell): Maxwell's equations in vacuum map TM^z
    onto TE^z by Ez -> Hz, (Hx, Hy) -> (-Ex, -Ey); the sources match too."""
    p = W.problem(nx=64, ny=48, radius=0.4, kind="homogeneous", eps1=1.0, wavelength=20.0, steps=700, avg_periods=1)
    mat = np.zeros((48, 64), np.uint8)
    tm = O.solve(p, mat=mat)
    te = O.solve(_te(p), mat=mat)
    assert np.abs(tm["ez"]).max() > 0.5
    np.testing.assert_allclose(te["ez"], tm["ez"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(te["hx"], -tm["hx"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(te["hy"], -tm["hy"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind,deg", [("homogeneous", 0.0), ("metallo_dielectric_janus", 90.0),
                                      ("dielectric_janus", 270.0)])
def test_te_zero_lift_and_torque_for_mirror_symmetric_bodies(kind, deg):
    p = _te(W.problem(nx=80, ny=80, radius=12.0, kind=kind, eps1=2.0, eps2=5.0, phi0_deg=deg, wavelength=24.0,
                      steps=1500))
    r = O.solve(p, fields=False)
    assert r["fx"] > 0.05
    assert abs(r["fy"]) < 1e-13 and abs(r["tz"]) < 1e-13


@pytest.mark.parametrize("kind,deg", [("metallo_dielectric_janus", 30.0), ("dielectric_janus", 200.0)])
def test_te_mirror_rule(kind, deg):
    p = _te(W.problem(nx=80, ny=80, radius=12.0, kind=kind, eps1=2.0, eps2=5.0, phi0_deg=deg, wavelength=24.0,
                      steps=1500))
    a = O.solve(p, fields=False)
    b = O.solve(dict(p, phi0=math.pi - p["phi0"]), fields=False)
    assert abs(a["fy"]) > 1e-3
    assert abs(a["fx"] - b["fx"]) < 1e-12 and abs(a["fy"] + b["fy"]) < 1e-12 and abs(a["tz"] + b["tz"]) < 1e-12


def test_te_norm_is_conserved_in_closed_boxes():
    """tau = 1/2 makes the collision a reflection in the norm with weights 1/w_q,
    w_q the field coefficient of the equilibrium (1/6 moving, 1/3 for the Hz
    rest, eps - 2/3 for the Ex and Ey rests); streaming only moves moving
    populations.  Conductor nodes (Ex = Ey = 0, the limit eps -> oo) drop the
    Ex and Ey rests, whose weights vanish; f -> f^eq(Hz(f), 0, 0) is the
    orthogonal projection for the remaining weights."""
    nx = ny = 48
    eps_of = np.array([1.0, 2.0, 4.0, 1.0])
    for kind, boundary in (("dielectric_janus", "periodic"), ("metallo_dielectric_janus", "pec_box")):
        p = _te(W.problem(nx=nx, ny=ny, radius=8.0, kind=kind, eps1=2.0, eps2=4.0, phi0_deg=30.0, wavelength=24.0,
                          steps=20000, avg_periods=0))
        mat = O.mask(p)
        if boundary == "pec_box":
            mat[0, :] = mat[-1, :] = mat[:, 0] = mat[:, -1] = O.MAT_PEC
        jj, ii = np.mgrid[0:ny, 0:nx]
        hz = np.exp(-((ii - 12.0) ** 2 + (jj - 30.0) ** 2) / 18.0)
        hz = np.where(mat == O.MAT_PEC, 0.0, hz)
        st = np.zeros((11, ny, nx))
        st[0] = hz / 3.0
        st[1:5] = hz / 6.0
        r = O.solve(p, boundary="periodic", mat=mat, state=st, energy=True)

        def norm(s):
            eps = eps_of[mat]
            moving = 6.0 * np.sum(s[[1, 2, 3, 4, 6, 7, 9, 10]] ** 2, axis=0)
            cond = mat == O.MAT_PEC
            rest = 3.0 * s[0] ** 2 + np.where(cond, 0.0, (s[5] ** 2 + s[8] ** 2) / np.where(cond, 1.0, eps - 2.0 / 3.0))
            return float(np.sum(moving + rest))

        n0, n1 = norm(st), norm(r["state"])
        assert abs(n1 - n0) / n0 < 1e-10
        w = r["energy"]
        assert w.max() / w.min() < 1.5


def test_te_dielectric_cylinder_matches_the_mie_series():
    """eps 2, a = 10, lambda = 40 (k0 a = pi / 2): drag within 1 %, far field within 5 % of its peak."""
    x = math.pi / 2
    c = A.mie_te_coeffs(x, 2.0, 0.0)
    fx = A.forces_closed_form(*c, x, 0.0)[0]
    r = O.solve(_te(W.config1()), fields=False, far_angles=72)
    assert abs(r["fx"] - fx) / fx < 0.01, (r["fx"], fx)
    assert abs(r["fy"]) < 1e-13 and abs(r["tz"]) < 1e-13
    B, D = A.scattering_coeffs(c[0], c[1], x, 0.0)
    phi = 2 * math.pi * np.arange(72) / 72
    ref = A.far_intensity(B, D, phi + math.pi)
    assert np.abs(r["s2"] - ref).max() < 0.05 * ref.max()


def test_te_conducting_cylinder_matches_the_series():
    """a / lambda = 0.5: drag within 5 % at a = 24 (Sec. III's bar); the far
    field's staircase error falls with resolution (18 % -> 11 % of the peak
    from a = 16 to 24: TE^z surface currents follow the staircase)."""
    x = math.pi
    c = A.pec_te_coeffs(x)
    fx = A.forces_closed_form(*c, x, 0.0)[0]
    B, D = A.scattering_coeffs(c[0], c[1], x, 0.0)
    phi = 2 * math.pi * np.arange(36) / 36
    ref = A.far_intensity(B, D, phi + math.pi)
    errs = []
    for a in (16, 24):
        p = _te(W.problem(nx=8 * a, ny=8 * a, radius=float(a), kind="homogeneous", eps1=1.0, wavelength=2.0 * a,
                          steps=W.steps_for(2.0 * a, 30), avg_periods=1))
        mat = O.mask(p)
        mat[mat == O.MAT_REGION2] = O.MAT_PEC
        r = O.solve(p, mat=mat, fields=False, far_angles=36)
        errs.append((abs(r["fx"] - fx) / fx, np.abs(r["s2"] - ref).max() / ref.max()))
    assert errs[1][0] < 0.05 and errs[1][0] < errs[0][0]
    assert errs[1][1] < 0.7 * errs[0][1]
