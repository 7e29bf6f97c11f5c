"""Pins of the oracle's instantaneous force trace and of an off-centre body
(arXiv 2509.22308, Sec. III: the forces settle into a steady oscillation at
twice the frequency of the incident wave, from the quadratic dependence of
the stress on the fields).  All run on the CPU."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


@pytest.mark.parametrize("case", ["mie", "mdjc"])
def test_force_trace_averages_to_the_force_and_oscillates_at_twice_the_frequency(case):
    p = W.config1() if case == "mie" else W.small_mdjc(4.0, 30.0, a=16)
    r = O.solve(p, fields=False, force_trace=True)
    f = r["force_trace"]
    T = int(round(3 * p["wavelength"]))
    window = p["avg_periods"] * T
    # the stress is linear in the time-averaged products: the mean of the
    # instantaneous forces over the window is the averaged force
    np.testing.assert_allclose(f[-window:].mean(axis=0), [r["fx"], r["fy"], r["tz"]], rtol=0, atol=1e-12)
    # steady state: periodic, with only the mean and the second harmonic
    assert np.abs(f[-T:] - f[-2 * T:-T]).max() < 1e-3
    for q in range(3):
        c = np.abs(np.fft.rfft(f[-T:, q])) / T
        if case == "mie" and q > 0:  # a symmetric body: no lift, no torque at any instant
            assert np.abs(f[:, q]).max() < 1e-12
            continue
        assert c[2] > 0.01 and c[1] < 1e-3 * c[2] and c[3] < 1e-3 * c[2], (q, c[:4])


def test_off_centre_body_by_whole_cells_keeps_its_forces():
    """A disk moved by whole cells has the same staircase (the material map is
    the shifted one, exactly); the incident wave is uniform in y and only
    changes phase along x, so the time-averaged forces agree up to the open
    edges' residual reflections, which reach the body differently: about 1 %
    on a 16a domain (a = 16)."""
    p = dict(W.small_mdjc(4.0, 30.0, a=16), nx=256, ny=256)
    c = (p["nx"] - 1) / 2
    moved = dict(p, cx=c + 7.0, cy=c - 5.0)
    m0, m1 = O.mask(p), O.mask(moved)
    assert np.array_equal(np.roll(np.roll(m0, -5, axis=0), 7, axis=1), m1)
    a = O.solve(p, fields=False)
    b = O.solve(moved, fields=False)
    for q in ("fx", "fy", "tz"):
        assert abs(a[q] - b[q]) < 0.02 * max(1.0, abs(a[q])), (q, a[q], b[q])
