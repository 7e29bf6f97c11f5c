"""Oracle of the overdamped particle motion of arXiv 2509.22308, Sec. IV.C.

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's
trajectory integrator; nothing in the product path imports it.

Sec. IV.C balances the radiation force and torque against the slender-body
Stokes resistance (Eqs. force-torque balance, hydro-force-torque) and, in the
non-dimensional variables x~ = x / a, t~ = t / T0 with T0 = a eta / F0,
arrives at
    dx~/dt~ = log(l/a) F~x(phi0) / (4 pi),
    dy~/dt~ = log(l/a) F~y(phi0) / (4 pi),
    dphi0/dt~ = M~z(phi0) / (2 pi).
Here F~x, F~y, M~z come from one row of a design map sampled at uniform
angles over one period; between samples they are the periodic cubic spline
(scipy's CubicSpline with periodic ends), and the system is integrated by
scipy's DOP853 at tight tolerances.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.interpolate import CubicSpline


def spline(phi_first: float, values) -> CubicSpline:
    v = np.asarray(values, dtype=np.float64)
    n = len(v)
    x = phi_first + 2 * math.pi * np.arange(n + 1) / n
    return CubicSpline(x, np.append(v, v[0]), bc_type="periodic")


def trajectory(phi_first: float, fx, fy, tz, phi_start: float, times, log_l_over_a: float = math.log(10.0),
               rtol: float = 1e-12, atol: float = 1e-12):
    """(x, y, phi) at the given times from (0, 0, phi_start)."""
    sx, sy, st = spline(phi_first, fx), spline(phi_first, fy), spline(phi_first, tz)
    period = 2 * math.pi
    cv = log_l_over_a / (4 * math.pi)

    def wrap(p):
        return phi_first + np.mod(p - phi_first, period)

    def rhs(_t, s):
        p = wrap(s[2])
        return [cv * sx(p), cv * sy(p), st(p) / (2 * math.pi)]

    times = np.asarray(times, dtype=np.float64)
    sol = solve_ivp(rhs, (0.0, float(times[-1])), [0.0, 0.0, float(phi_start)], method="DOP853", t_eval=times,
                    rtol=rtol, atol=atol)
    if not sol.success:
        raise RuntimeError(sol.message)
    return sol.y[0], sol.y[1], sol.y[2]
