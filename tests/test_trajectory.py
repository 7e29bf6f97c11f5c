"""Trajectories of Sec. IV.C (arXiv 2509.22308): the oracle pinned to closed
forms, and the library's host-side integrator (jlb_trajectory, no device
work) against the oracle.  All run on the CPU."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import paper_2509_22308_amd as J
from oracle import trajectory as TR

N = 180
PHI = 2 * math.pi * np.arange(N) / N
CV = math.log(10.0) / (4 * math.pi)


def _sinusoidal_map(A=0.5, star=1.0):
    fx = 1.0 + 0.3 * np.cos(PHI)
    fy = 0.2 * np.sin(2 * PHI)
    tz = -A * np.sin(PHI - star)
    return fx, fy, tz


def _closed_phi(t, p0, A=0.5, star=1.0):
    """dphi/dt = -(A / 2 pi) sin(phi - phi*): tan((phi - phi*)/2) decays as exp(-A t / 2 pi)."""
    return star + 2 * np.arctan(np.tan((p0 - star) / 2) * np.exp(-A * t / (2 * math.pi)))


def test_oracle_orientation_follows_the_closed_form_and_reaches_the_attractor():
    fx, fy, tz = _sinusoidal_map()
    t = np.array([0.0, 10.0, 100.0, 1000.0, 10000.0])
    for p0 in (0.0, math.pi / 4, 7 * math.pi / 6 - 2 * math.pi):
        x, y, p = TR.trajectory(0.0, fx, fy, tz, p0, t)
        # phi is unwrapped, the closed form lives on one branch: compare modulo 2 pi
        np.testing.assert_allclose(np.angle(np.exp(1j * (p - _closed_phi(t, p0)))), 0.0, atol=1e-7)
        assert abs(np.angle(np.exp(1j * (p[-1] - 1.0)))) < 1e-9  # the torque-free angle with negative slope attracts
        # positions by quadrature of the closed-form orientation (a route without the ODE solver);
        # the spline through 180 samples differs from the sinusoids by ~1e-8
        for k in (2, 3):
            xq = quad(lambda s: CV * (1.0 + 0.3 * math.cos(_closed_phi(s, p0))), 0, t[k], limit=400)[0]
            yq = quad(lambda s: CV * 0.2 * math.sin(2 * _closed_phi(s, p0)), 0, t[k], limit=400)[0]
            assert abs(x[k] - xq) < 2e-8 * t[k] and abs(y[k] - yq) < 2e-8 * t[k], (k, x[k] - xq, y[k] - yq)


def test_oracle_torque_free_motion_is_a_straight_line():
    fx = 1.0 + 0.3 * np.cos(PHI)
    fy = 0.4 * np.sin(PHI)
    tz = np.zeros(N)
    t = np.array([0.0, 500.0, 10000.0])
    x, y, p = TR.trajectory(0.0, fx, fy, tz, PHI[30], t)
    np.testing.assert_allclose(x, CV * fx[30] * t, rtol=1e-12)
    np.testing.assert_allclose(y, CV * fy[30] * t, rtol=1e-12)


def _random_row(seed):
    rng = np.random.default_rng(seed)
    def series(scale, mean=0.0):
        v = np.full(N, mean)
        for m in range(1, 7):
            v += scale / m ** 2 * (rng.normal() * np.cos(m * PHI) + rng.normal() * np.sin(m * PHI))
        return v
    return series(0.4, 1.5), series(0.5), series(0.3)


def _lib(fx, fy, tz, p0, t_end=1e4, dt=0.5, every=2000, phi_first=0.0):
    from paper_2509_22308_amd.maps import trajectory
    return trajectory(phi_first + PHI, fx, fy, tz, p0, t_end=t_end, dt=dt, record_every=every)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("p0", [0.0, math.pi / 4, 7 * math.pi / 6])
def test_library_trajectory_matches_the_oracle(seed, p0):
    fx, fy, tz = _random_row(seed)
    t, x, y, p = _lib(fx, fy, tz, p0)
    xo, yo, po = TR.trajectory(0.0, fx, fy, tz, p0, t)
    scale = max(1.0, np.abs(xo).max())
    assert np.abs(x - xo).max() < 1e-7 * scale and np.abs(y - yo).max() < 1e-7 * scale
    assert np.abs(p - po).max() < 1e-8


def test_library_spline_is_the_periodic_cubic_spline():
    """Zero torque freezes phi0, so x / (c t) reads the interpolant at phi0:
    exact at the samples, scipy's periodic spline between them, across the seam."""
    fx, fy, _ = _random_row(7)
    tz = np.zeros(N)
    ref = TR.spline(0.3, fx)
    for p0 in (0.3 + PHI[17], 0.3 + 0.5 * (PHI[17] + PHI[18]), 0.3 - 0.01, 0.3 + 2 * math.pi * 5.37):
        t, x, y, p = _lib(fx, fy, tz, p0, t_end=10.0, dt=1.0, every=10, phi_first=0.3)
        wrapped = 0.3 + (p0 - 0.3) % (2 * math.pi)
        assert abs(x[-1] / (CV * 10.0) - ref(wrapped)) < 1e-12
        assert p[-1] == p0
    t, x, y, p = _lib(fx, fy, tz, 0.3 + PHI[17], t_end=10.0, dt=1.0, every=10, phi_first=0.3)
    assert abs(x[-1] - CV * 10.0 * fx[17]) < 1e-12


def test_library_rk4_converges_at_fourth_order():
    fx, fy, tz = _sinusoidal_map(A=3.0, star=2.0)
    t_end = 40.0
    exact = _closed_phi(t_end, 0.2, A=3.0, star=2.0)
    errs = []
    for dt in (2.0, 1.0, 0.5):
        t, x, y, p = _lib(fx, fy, tz, 0.2, t_end=t_end, dt=dt, every=int(round(t_end / dt)))
        errs.append(abs(p[-1] - exact))
    # the spline's own error (~1e-8 for 180 samples of a sinusoid) floors the sequence
    assert errs[0] / errs[1] > 10 and errs[1] > errs[2]


def test_trajectory_argument_errors():
    lib = J.load()
    a = np.zeros(N)
    out = np.zeros(8)
    ptr = lambda v: J._vp(v.ctypes.data)  # noqa: E731
    assert lib.jlb_trajectory(3, 0.0, ptr(a), ptr(a), ptr(a), 0.0, 0.5, 1, 1.0, 1, ptr(out)) == -1
    assert lib.jlb_trajectory(N, 0.0, None, ptr(a), ptr(a), 0.0, 0.5, 1, 1.0, 1, ptr(out)) == -1
    assert lib.jlb_trajectory(N, 0.0, ptr(a), ptr(a), ptr(a), 0.0, 0.0, 1, 1.0, 1, ptr(out)) == -1
    assert lib.jlb_trajectory(N, 0.0, ptr(a), ptr(a), ptr(a), 0.0, 0.5, 1, 1.0, 0, ptr(out)) == -1
    b = a.copy()
    b[5] = np.nan
    assert lib.jlb_trajectory(N, 0.0, ptr(b), ptr(a), ptr(a), 0.0, 0.5, 1, 1.0, 1, ptr(out)) == -1
    assert "non-finite" in J.jlb_last_error()
