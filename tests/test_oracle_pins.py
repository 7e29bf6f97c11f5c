"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test holds it to a closed
form, an exact invariant, a textbook series or a value printed in
arXiv 2509.22308.  All run on the CPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as W
from oracle import analytic as A
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Geometry: Sec. II, Fig. (schematic); orientation from Sec. IV.A.2 / App. A
# ----------------------------------------------------------------------------

def test_mask_regions_follow_the_papers_orientation_words():
    base = dict(nx=64, ny=64, radius=20.0, kind="metallo_dielectric_janus", eps1=2.0, wavelength=40.0, steps=0)
    c = 31.5
    # phi0 = pi/2: dielectric half faces the incident wave, which comes from the left (Sec. IV.A.2)
    m = O.mask(W.problem(phi0=math.pi / 2, **base))
    assert m[32, int(c - 10)] == O.MAT_REGION2 and m[32, int(c + 10)] == O.MAT_PEC
    # phi0 = 3 pi / 2: PEC half faces the wave
    m = O.mask(W.problem(phi0=3 * math.pi / 2, **base))
    assert m[32, int(c - 10)] == O.MAT_PEC and m[32, int(c + 10)] == O.MAT_REGION2
    # phi0 = 0: PEC half along +y (App. A)
    m = O.mask(W.problem(phi0=0.0, **base))
    assert m[int(c + 10), 32] == O.MAT_PEC and m[int(c - 10), 32] == O.MAT_REGION2


def test_mask_staircase_and_tie_rule():
    p = W.problem(nx=40, ny=40, radius=10.0, kind="dielectric_janus", eps1=2.0, eps2=3.0, phi0_deg=45.0,
                  wavelength=40.0, steps=0)
    m = O.mask(p)
    jj, ii = np.mgrid[0:40, 0:40]
    dx, dy = ii - 19.5, jj - 19.5
    inside = dx * dx + dy * dy <= 100.0
    assert np.array_equal(m > 0, inside)
    s = -dx * math.sin(math.pi / 4) - dy * math.cos(math.pi / 4)
    assert np.array_equal(m[inside & (s > 1e-9)], np.full(np.sum(inside & (s > 1e-9)), 1))
    # cells on the diagonal interface (dx = -dy) tie and belong to region III
    tie = inside & (np.abs(dx + dy) < 1e-12)
    assert tie.sum() > 0 and np.all(m[tie] == O.MAT_REGION3)
    # homogeneous: every inside node is region II
    p["kind"] = "homogeneous"
    assert np.array_equal(O.mask(p) == 1, inside)


# ----------------------------------------------------------------------------
# Lattice: plane-wave phase speed and the discrete dispersion relation
# ----------------------------------------------------------------------------

def _strip(eps, lam=40.0, nx=800, steps=4000, pec_from=None):
    """Fields along a 1-row strip at two times a quarter period apart."""
    T = int(round(3 * lam))
    p = W.problem(nx=nx, ny=1, radius=0.0, kind="homogeneous", eps1=eps, wavelength=lam, steps=steps,
                  avg_periods=0)
    mat = np.full((1, nx), 1 if eps != 1.0 else 0, np.uint8)
    if pec_from is not None:
        mat[:, pec_from:] = O.MAT_PEC
    r1 = O.solve(p, mat=mat, boundary="x_open_y_periodic")
    p2 = dict(p, steps=steps + T // 4)
    r2 = O.solve(p2, mat=mat, boundary="x_open_y_periodic")
    return r1["ez"][0], r2["ez"][0]


def _vacuum_k(omega):
    # right-going branch of the D3Q7 tau = 1/2 model in vacuum:
    # sin(omega - k/2) = -(1/3) sin(k/2)  <=>  k = omega + 2 atan(2 tan(omega/2))
    return omega + 2.0 * math.atan(2.0 * math.tan(omega / 2.0))


def _dielectric_k(omega, eps):
    # implicit relation for propagation along x in a uniform medium eps:
    # [(B - A) + (6 eps - 2) C] [(B - A) + 4 C] = (A + B)^2,
    # A = tan((k - omega)/2), B = tan((k + omega)/2), C = tan(omega/2)
    def f(k):
        a, b, c = math.tan((k - omega) / 2), math.tan((k + omega) / 2), math.tan(omega / 2)
        return ((b - a) + (6 * eps - 2) * c) * ((b - a) + 4 * c) - (a + b) ** 2
    kc = 3.0 * math.sqrt(eps) * omega
    return brentq(f, 0.8 * kc, 1.2 * kc)


@pytest.mark.parametrize("eps", [1.0, 2.0, 4.0])
def test_plane_wave_phase_speed_matches_lattice_dispersion(eps):
    lam = 40.0
    omega = 2 * math.pi / (3 * lam)
    e1, e2 = _strip(eps, lam)
    theta = np.unwrap(np.arctan2(e1, e2))
    xs = np.arange(100, 600)
    k_meas = -np.polyfit(xs, theta[xs], 1)[0]
    k_lat = _vacuum_k(omega) if eps == 1.0 else _dielectric_k(omega, eps)
    k_cont = 3.0 * math.sqrt(eps) * omega  # continuum: phase speed 1/(3 sqrt(eps))
    assert abs(k_meas - k_lat) / k_lat < 1e-6
    # the lattice value is distinguishable from the continuum one at this resolution
    assert abs(k_cont - k_lat) / k_lat > 4e-4
    # free-space phase speed -> 1/3 cell per step
    if eps == 1.0:
        assert abs(omega / k_meas - 1.0 / 3.0) < 2e-4


def test_open_boundary_reflection_below_papers_level():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        rmax = json.load(f)["open_boundary"]["reflection_max"]
    # normal incidence on the right edge of a vacuum domain (the edges of every
    # problem here are vacuum); the entering population of an outgoing wave vanishes
    e1, e2 = _strip(1.0)
    amp = np.hypot(e1, e2)[100:600]
    refl = (amp.max() - amp.min()) / (amp.max() + amp.min())
    assert refl < rmax * 1e-3, refl
    # the injected amplitude differs from E0 only by the O((k dx)^2) source error
    e1, e2 = _strip(1.0)
    assert abs(np.hypot(e1, e2)[100:600].mean() - 1.0) < 3e-3


def _wall_fit(lam, nx, steps):
    """Standing wave in front of a conductor filling x >= nx - 100: the fitted
    wall position x_w, amplitude / (2 E_inc) and the largest fit residual of
    |E| = A |sin(k (x - x_w))| over seven wavelengths in front of it."""
    from scipy.optimize import minimize_scalar
    pf = nx - 100
    e1, e2 = _strip(1.0, lam, nx=nx, steps=steps, pec_from=pf)
    amp = np.hypot(e1, e2)
    k = _vacuum_k(2 * math.pi / (3 * lam))
    xs = np.arange(pf - int(7 * lam), pf - 10)

    def fit(xw):
        model = np.abs(np.sin(k * (xs - xw)))
        a = np.dot(model, amp[xs]) / np.dot(model, model)
        return a, np.max(np.abs(amp[xs] - a * model))

    r = minimize_scalar(lambda xw: fit(xw)[1], bounds=(pf - 2.0, pf + 1.0), method="bounded",
                        options={"xatol": 1e-9})
    a, res = fit(r.x)
    return r.x - pf, a / 2.0, res


def test_open_top_and_bottom_edges_pass_the_plane_wave_exactly():
    """Sec. III: the wave enters on the left and the other edges let outgoing
    waves leave.  The incident plane wave is uniform in y, so in an empty
    domain every row must equal the solution of a domain periodic in y: the
    top and bottom edges (extrapolation relaxed against the companion row)
    must not disturb it at all."""
    nx, ny = 300, 40
    p = W.problem(nx=nx, ny=ny, radius=2.0, kind="homogeneous", eps1=1.0, wavelength=40.0, steps=1500,
                  avg_periods=0)
    mat = np.zeros((ny, nx), np.uint8)
    r = O.solve(p, mat=mat)
    rp = O.solve(p, mat=mat, boundary="x_open_y_periodic")
    scale = np.abs(rp["ez"]).max()
    assert scale > 0.9
    for f in ("ez", "hx", "hy"):
        assert np.abs(r[f] - rp[f]).max() <= 1e-13 * scale, f


def _edge_pulse(ny, steps, nx=200, x0=100.0, y0=90.0, sigma=4.0):
    """A Gaussian E_z pulse (equilibrium, H = 0) in an empty domain with open
    edges and no incident wave."""
    jj, ii = np.mgrid[0:ny, 0:nx]
    ez = np.exp(-((ii - x0) ** 2 + (jj - y0) ** 2) / (2 * sigma ** 2))
    st = np.zeros((11, ny, nx))
    st[0] = (1.0 - 2.0 / 3.0) * ez
    st[1:5] = ez / 6.0
    p = W.problem(nx=nx, ny=ny, radius=2.0, kind="homogeneous", eps1=1.0, wavelength=40.0, steps=steps,
                  avg_periods=0, ramp_periods=0, e0=1e-300)
    return O.solve(p, mat=np.zeros((ny, nx), np.uint8), state=st)


@pytest.mark.parametrize("steps", [200, 260])
def test_open_edge_reflects_no_more_than_a_first_order_absorbing_edge(steps):
    """Sec. III: first-order extrapolation at the open edges, residual
    reflections small.  A pulse 29.5 cells below the top edge sends rays at
    every incidence angle up to theta_max = acos(29.5 / (steps / 3)); the
    energy the edge sends back (this domain minus one whose top edge lies
    300 rows further up) is at most what the first-order absorbing edge of
    Engquist and Majda reflects, amplitude tan^2(theta / 2), for rays spread
    evenly over those angles.  Normal incidence alone reflects nothing
    (test_open_boundary_reflection_below_papers_level)."""
    a, b = _edge_pulse(120, steps), _edge_pulse(420, steps)
    refl = 0.5 * sum(np.sum((a[f] - b[f][:120]) ** 2) for f in ("ez", "hx", "hy"))
    crossed = 0.5 * sum(np.sum(b[f][120:] ** 2) for f in ("ez", "hx", "hy"))
    tmax = math.acos((119.5 - 90.0) / (steps / 3.0))
    th = np.linspace(0.0, tmax, 4001)
    em1 = np.trapezoid(np.tan(th / 2.0) ** 4, th) / tmax
    assert crossed > 0.3 * 0.5 * sum(np.sum(b[f] ** 2) for f in ("ez", "hx", "hy"))
    assert refl / crossed < em1, (refl / crossed, em1)


def test_energy_weights_the_electric_field_by_eps():
    """The energy diagnostic (Sec. III: the total field energy approaches a
    constant) is W = sum (eps E_z^2 + H^2) / 2.  A standing wave in a
    periodic uniform eps = 4 box trades electric for magnetic energy every
    quarter period; only with the electric part weighted by eps is W
    constant (here to the lattice's O((k dx)^2) = 1e-2 level: 1.5e-3 over
    four periods).  Without the weight, W would swing by (eps - 1) / (eps + 1)
    = 60 %."""
    n, eps, lam = 128, 4.0, 64.0
    k = 2 * math.pi / lam
    ii = np.mgrid[0:8, 0:n][1]
    ez = np.cos(k * ii)
    st = np.zeros((11, 8, n))
    st[0] = (eps - 2.0 / 3.0) * ez
    st[1:5] = ez / 6.0
    period = 3.0 * math.sqrt(eps) * lam
    p = W.problem(nx=n, ny=8, radius=2.0, kind="homogeneous", eps1=eps, wavelength=40.0, steps=int(4 * period),
                  avg_periods=0, ramp_periods=0, e0=1e-300)
    w = O.solve(p, boundary="periodic", mat=np.full((8, n), 1, np.uint8), state=st, energy=True, fields=False)["energy"]
    assert (w.max() - w.min()) / w.mean() < 5e-3
    # the electric energy at t = 0 reappears as magnetic energy a quarter period later
    assert abs(w[0] - 0.5 * eps * np.sum(ez ** 2)) / w[0] < 5e-3


def test_flat_conductor_wall_reflects_totally():
    """Sec. II: E_z = 0 on the conductor.  A plane wave meeting a flat
    conductor (conductor nodes from x = x_c on) reflects totally: in front of
    it |E| is a pure standing wave 2 E_inc |sin(k (x - x_w))| (amplitude
    within the source's O((k dx)^2) error of 2, no travelling part).  Its node
    x_w sits between the last open node's link midpoint and the first
    conductor node, at the same place for every wavelength (a wall, not a
    frequency-dependent phase)."""
    w40, a40, r40 = _wall_fit(40.0, 800, 4000)
    w80, a80, r80 = _wall_fit(80.0, 1400, 8000)
    assert r40 < 1e-5 and r80 < 1e-5, (r40, r80)
    assert abs(a40 - 1.0) < 3e-3 and abs(a80 - 1.0) < 1e-3, (a40, a80)
    assert -0.5 < w40 <= 0.0 and abs(w80 - w40) < 1e-3, (w40, w80)


# ----------------------------------------------------------------------------
# Lattice: the printed update as a matrix, eigenmodes on a periodic grid
# ----------------------------------------------------------------------------

_C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)


def _literal_symbol(k, eps):
    """42 x 42 Fourier symbol of post-collision state -> next post-collision state.

    State order [e/h][velocity i][component]; Eq. (LBGK equation) with the
    equilibria of Eq. (equilibrium distribution functions), mu_r = 1.
    """
    n = 42

    def eq_of(s):
        e = s[:21].reshape(7, 3)
        h = s[21:].reshape(7, 3)
        E = e.sum(0) / eps
        H = h.sum(0)
        ee = np.empty((7, 3))
        he = np.empty((7, 3))
        ee[0] = (eps - 1.0) * E
        he[0] = 0.0 * H
        for i in range(1, 7):
            ee[i] = (E - np.cross(_C[i], H)) / 6.0
            he[i] = (H + np.cross(_C[i], E)) / 6.0
        return np.concatenate([ee.ravel(), he.ravel()])

    Q = np.stack([eq_of(u) for u in np.eye(n)], axis=1)
    coll = 2.0 * Q - np.eye(n)
    phase = np.exp(-1j * (_C[:, 0] * k[0] + _C[:, 1] * k[1]))
    S = np.diag(np.concatenate([np.repeat(phase, 3), np.repeat(phase, 3)]))
    return coll @ S


def test_printed_update_is_non_dissipative_and_has_maxwell_long_wave_limit():
    for eps in (1.0, 2.5, 10.0):
        for ang in (0.0, 0.4, math.pi / 4, 1.2):
            kk = 0.02
            G = np.linalg.eigvals(_literal_symbol((kk * math.cos(ang), kk * math.sin(ang)), eps))
            assert np.allclose(np.abs(G), 1.0, atol=1e-9)
            # slowest non-trivial branch: phase speed 1/(3 sqrt(eps)) (Maxwell in a medium)
            w = np.abs(np.angle(G))
            w = w[w > 1e-6]
            c = w.min() / kk
            assert abs(c - 1.0 / (3.0 * math.sqrt(eps))) < 2e-3 / math.sqrt(eps)


def test_vacuum_dispersion_closed_form_is_an_eigenvalue_of_the_printed_update():
    for lam in (40.0, 96.0, 128.0):
        omega = 2 * math.pi / (3 * lam)
        G = np.linalg.eigvals(_literal_symbol((_vacuum_k(omega), 0.0), 1.0))
        assert np.min(np.abs(G - np.exp(-1j * omega))) < 1e-12


@pytest.mark.parametrize("eps,mk", [(1.0, (3, 2)), (2.5, (1, 5)), (7.0, (4, 0))])
def test_oracle_literal_mode_evolves_eigenmodes_exactly(eps, mk):
    nx, ny = 32, 24
    k = (2 * math.pi * mk[0] / nx, 2 * math.pi * mk[1] / ny)
    G, V = np.linalg.eig(_literal_symbol(k, eps))
    # a travelling (non-real) mode with field content
    score = np.abs(V[20, :]) + np.abs(V[21 + 0, :]) * 0 + np.where(np.abs(np.imag(G)) > 1e-6, 1.0, 0.0)
    j = int(np.argmax(score))
    v, g = V[:, j], G[j]
    jj, ii = np.mgrid[0:ny, 0:nx]
    ph = np.exp(1j * (k[0] * ii + k[1] * jj))
    st0 = np.real(v[:, None, None] * ph).reshape(2, 7, 3, ny, nx)
    n = 60
    p = W.problem(nx=nx, ny=ny, radius=0.0, kind="homogeneous", eps1=eps, wavelength=40.0, steps=n,
                  avg_periods=0)
    mat = np.full((ny, nx), 1 if eps != 1.0 else 0, np.uint8)
    r = O.solve(p, literal=True, boundary="periodic", mat=mat, state=st0)
    expect = np.real(v[:, None, None] * g ** n * ph).reshape(2, 7, 3, ny, nx)
    assert np.max(np.abs(r["state"] - expect)) < 1e-12 * max(1.0, np.max(np.abs(expect)))


# ----------------------------------------------------------------------------
# Literal (printed) equations == reduced 11-population form
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["homogeneous", "dielectric_janus", "metallo_dielectric_janus"])
def test_literal_and_reduced_modes_agree(kind):
    p = W.problem(nx=72, ny=66, radius=12.0, kind=kind, eps1=3.0, eps2=6.5, phi0_deg=37.0, wavelength=24.0,
                  steps=900, avg_periods=2)
    a = O.solve(p, literal=False)
    b = O.solve(p, literal=True)
    scale = max(np.max(np.abs(a["ez"])), np.max(np.abs(a["hy"])))
    for f in ("ez", "hx", "hy"):
        assert np.max(np.abs(a[f] - b[f])) <= 1e-13 * scale
    for q in ("fx", "fy", "tz"):
        assert abs(a[q] - b[q]) <= 1e-12 * max(1.0, abs(a[q]))


# ----------------------------------------------------------------------------
# Symmetry laws: Sec. IV.A.2 / IV.B.1, exact to rounding
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind,deg", [("homogeneous", 0.0), ("metallo_dielectric_janus", 90.0),
                                      ("metallo_dielectric_janus", 270.0), ("dielectric_janus", 90.0),
                                      ("dielectric_janus", 270.0)])
def test_zero_lift_and_torque_for_mirror_symmetric_bodies(kind, deg):
    p = W.problem(nx=80, ny=80, radius=12.0, kind=kind, eps1=2.0, eps2=5.0, phi0_deg=deg, wavelength=24.0,
                  steps=1500)
    r = O.solve(p, fields=False)
    assert r["fx"] > 0.1
    assert abs(r["fy"]) < 1e-13 and abs(r["tz"]) < 1e-13


@pytest.mark.parametrize("kind,deg", [("metallo_dielectric_janus", 30.0), ("dielectric_janus", 45.0),
                                      ("metallo_dielectric_janus", 45.0), ("dielectric_janus", 200.0)])
def test_mirror_rule_phi0_to_pi_minus_phi0(kind, deg):
    p = W.problem(nx=80, ny=80, radius=12.0, kind=kind, eps1=2.0, eps2=5.0, phi0_deg=deg, wavelength=24.0,
                  steps=1500)
    q = dict(p, phi0=math.pi - p["phi0"])
    a = O.solve(p, fields=False)
    b = O.solve(q, fields=False)
    assert abs(a["fy"]) > 1e-3
    assert abs(a["fx"] - b["fx"]) < 1e-12
    assert abs(a["fy"] + b["fy"]) < 1e-12
    assert abs(a["tz"] + b["tz"]) < 1e-12


# ----------------------------------------------------------------------------
# Energy conservation with absorption neglected
# ----------------------------------------------------------------------------

def _pulse_state(nx, ny, x0, y0, width, mat, eps_of):
    """Equilibrium populations (reduced layout) of a Gaussian E_z pulse, H = 0."""
    jj, ii = np.mgrid[0:ny, 0:nx]
    ez = np.exp(-((ii - x0) ** 2 + (jj - y0) ** 2) / (2 * width ** 2))
    eps = eps_of[mat]
    ez = np.where(mat == O.MAT_PEC, 0.0, ez)
    st = np.zeros((11, ny, nx))
    st[0] = (eps - 2.0 / 3.0) * ez
    st[1:5] = ez / 6.0
    return st


def _weighted_norm(st, mat, eps_of):
    """Quadratic form conserved exactly by the update in a closed domain.

    With tau = 1/2 the collision is f -> 2 f^eq - f.  The map f -> f^eq is an
    orthogonal projection for the weights 1/w_q, where w_q is the coefficient
    of the field in the equilibrium (1/6 for the moving populations,
    eps - 2/3 for the rest e-population, 1/3 for the rest h-populations), so
    the collision is a reflection in that norm; streaming only moves moving
    populations, which all weigh 6.  A conductor node is the limit eps -> oo:
    its rest e-population weighs 1 / (eps - 2/3) -> 0 and drops out, and
    f -> f^eq(E = 0, H(f)) is the orthogonal projection for the remaining
    weights, so its collision is a reflection too.
    """
    eps = eps_of[mat]
    cond = mat == O.MAT_PEC
    moving = 6.0 * np.sum(st[[1, 2, 3, 4, 6, 7, 9, 10]] ** 2, axis=0)
    rest_h = 3.0 * st[5] ** 2 + 3.0 * st[8] ** 2
    rest_e = np.where(cond, 0.0, st[0] ** 2 / np.where(cond, 1.0, eps - 2.0 / 3.0))
    return float(np.sum(moving + rest_h + rest_e))


def test_energy_is_conserved_in_closed_boxes():
    """Lossless media: no energy is created or destroyed without open edges."""
    nx = ny = 48
    # periodic box with a dielectric Janus body, and a PEC-walled box with a metallo-dielectric one
    for kind, boundary in (("dielectric_janus", "periodic"), ("metallo_dielectric_janus", "pec_box")):
        p = W.problem(nx=nx, ny=ny, radius=8.0, kind=kind, eps1=2.0, eps2=4.0, phi0_deg=30.0, wavelength=24.0,
                      steps=20000, avg_periods=0)
        mat = O.mask(p)
        if boundary == "pec_box":
            mat[0, :] = mat[-1, :] = mat[:, 0] = mat[:, -1] = O.MAT_PEC
        eps_of = np.array([1.0, 2.0, 4.0, 1.0])
        st = _pulse_state(nx, ny, 12.0, 30.0, 3.0, mat, eps_of)
        r = O.solve(p, boundary="periodic", mat=mat, state=st, energy=True)
        n0 = _weighted_norm(st, mat, eps_of)
        n1 = _weighted_norm(r["state"], mat, eps_of)
        assert abs(n1 - n0) / n0 < 1e-10
        # the field energy (eps E^2 + H^2)/2 only trades with the non-equilibrium part: bounded, no growth
        w = r["energy"]
        assert w.max() / w.min() < 1.5
        assert w[-2000:].mean() < 1.05 * w[:2000].mean()


def test_driven_energy_reaches_a_plateau():
    # Sec. III: total energy approaches a constant; compare consecutive period means
    p = W.config1()
    r = O.solve(p, energy=True, fields=False)
    w = r["energy"]
    T = 120
    m1 = w[-2 * T:-T].mean()
    m2 = w[-T:].mean()
    assert abs(m2 - m1) / m2 < 2e-3


# ----------------------------------------------------------------------------
# Whole solves against closed-form physics
# ----------------------------------------------------------------------------

def _golden():
    with open(os.path.join(GOLDEN, "analytic_forces.json")) as f:
        return json.load(f)


def test_config1_homogeneous_cylinder_matches_mie_series():
    x = math.pi / 2  # a = 10, lambda = 40
    c = A.mie_coeffs(x, 2.0, 0.0)
    fx_mie = A.forces_closed_form(*c, x, 0.0)[0]
    r = O.solve(W.config1(), fields=False)
    assert abs(r["fx"] - fx_mie) / fx_mie < 0.02
    assert abs(r["fy"]) < 1e-13 and abs(r["tz"]) < 1e-13


@pytest.mark.parametrize("eps", [1.0, 3.0])
def test_diagonal_conductor_wall_keeps_the_field_energy(eps):
    """Sec. II: a perfect conductor reflects without loss, whatever the wall's
    angle to the lattice.  A smooth E_z pulse in a closed conductor box cut by
    a 45 degree conductor wall (a pure diagonal staircase) keeps its field
    energy: never below 0.9 of the start, as with an axis-aligned wall.  A
    link-wise reflection at such stair corners feeds the lattice's undamped
    non-equilibrium modes instead (field energy down to 0.32 in vacuum and
    0.62 at eps = 3 in this box)."""
    n = 96
    for angle in (0.0, 45.0):
        mat = np.full((n, n), 1, np.uint8)
        mat[0, :] = mat[-1, :] = mat[:, 0] = mat[:, -1] = O.MAT_PEC
        t = math.radians(angle)
        jj, ii = np.mgrid[0:n, 0:n]
        c = (n - 1) / 2
        mat[-(ii - c) * math.sin(t) + (jj - c) * math.cos(t) < -1e-9] = O.MAT_PEC
        eps_of = np.array([1.0, eps, 1.0, 1.0])
        st = _pulse_state(n, n, 0.35 * n, 0.62 * n, 4.0, mat, eps_of)
        p = W.problem(nx=n, ny=n, radius=2.0, kind="homogeneous", eps1=eps, wavelength=40.0, steps=6000,
                      avg_periods=0, ramp_periods=0, e0=1e-300)
        w = O.solve(p, boundary="periodic", mat=mat, state=st, energy=True, fields=False)["energy"]
        assert w.min() / w[0] > 0.9, (eps, angle, w.min() / w[0])


def test_no_scatterer_feels_no_force():
    """The degenerate body: eps = 1 everywhere.  The incident wave is then the
    whole field, the averaged stress on the contour has no net flux (Sec.
    II.B), and every force and the torque vanish to rounding."""
    for a in (10, 20):
        p = W.problem(nx=8 * a, ny=8 * a, radius=float(a), kind="homogeneous", eps1=1.0, wavelength=2.0 * a,
                      steps=W.steps_for(2.0 * a, 20), avg_periods=5)
        r = O.solve(p, fields=False)
        assert abs(r["fx"]) < 1e-12 and abs(r["fy"]) < 1e-12 and abs(r["tz"]) < 1e-12, (a, r)


def test_homogeneous_pec_cylinder_matches_series():
    """Textbook PEC series vs the oracle at a = 24, lambda = 48: the staircase
    error falls with the radius (4.9 %, 2.1 %, 2.4 %, 1.2 % at a = 8, 16, 24,
    32); Sec. III quotes 5 % for lambda / dx >= 10."""
    a = 24
    p = W.problem(nx=8 * a, ny=8 * a, radius=float(a), kind="homogeneous", eps1=1.0, wavelength=2.0 * a,
                  steps=W.steps_for(2.0 * a, 30))
    mat = O.mask(p)
    mat[mat == O.MAT_REGION2] = O.MAT_PEC
    r = O.solve(p, mat=mat, fields=False)
    x = math.pi
    fx = A.forces_closed_form(*A.pec_coeffs(x), x, 0.0)[0]
    assert abs(r["fx"] - fx) / fx < 0.05


@pytest.mark.parametrize("eps1,deg", [(2.0, 0.0), (2.0, 30.0), (4.0, 30.0), (8.0, 0.0), (8.0, 30.0),
                                      (1.5, 270.0)])
def test_metallo_dielectric_janus_matches_papers_analytic_solution(eps1, deg):
    """Sec. IV.A: the paper's analytic MDJC force/torque vs the lattice oracle.

    a = 24 cells at a / lambda = 0.5 (lambda / dx = 48).  Sec. III quotes 5 %
    on forces for lambda / dx >= 10; Sec. IV.A.2 notes larger relative errors
    where lift and torque are small, so those are held to an absolute band of
    0.03 (3 % of their full scale, 1.0 and 0.56) plus 5 % of the value.
    """
    ref = [g for g in _golden()["mdjc"] if abs(g["x"] - math.pi) < 1e-12 and g["eps1"] == eps1
           and g["phi0_deg"] == deg][0]
    r = O.solve(W.small_mdjc(eps1, deg, a=24), fields=False)
    assert abs(r["fx"] - ref["fx"]) / ref["fx"] < 0.05, (r["fx"], ref["fx"])
    for q in ("fy", "tz"):
        assert abs(r[q] - ref[q]) < 0.03 + 0.05 * abs(ref[q]), (q, r[q], ref[q])
