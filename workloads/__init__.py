"""Seeded synthetic workloads for the Janus-cylinder EM lattice Boltzmann solve.

This module holds parameters only (geometry, permittivities, orientation,
wavelength, grid, steps) and the seeded draws that pick them; it contains none
of the method's arithmetic, so the HIP library, the oracle and the benchmark
can all take their inputs from here.

Problem dicts use these keys (angles in radians under ``phi0``):
  nx, ny, radius, kind ('homogeneous' | 'dielectric_janus' |
  'metallo_dielectric_janus'), eps1, eps2, phi0, wavelength, e0, steps,
  avg_periods, ramp_periods, contour_offset, contour_points.

The paper (arXiv 2509.22308) uses no dataset: its force maps are parameter
sweeps (Sec. IV.A, Fig. HS75_Map; Sec. IV.B, Fig. 2D_map), so the sweeps below
are the workloads themselves, at the sizes the measurement plan names.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(e0=1.0, avg_periods=5, ramp_periods=1, contour_offset=3.0, contour_points=0)


def problem(**kw) -> dict:
    p = dict(DEFAULTS)
    if "phi0_deg" in kw:
        kw = dict(kw)
        kw["phi0"] = math.radians(kw.pop("phi0_deg"))
    p.update(kw)
    p.setdefault("phi0", 0.0)
    p.setdefault("eps2", 1.0)
    p.setdefault("ny", p["nx"])
    return p


def steps_for(wavelength: float, periods: int = 52) -> int:
    """Whole periods of T = 3 lambda steps (vacuum wave speed 1/3 cell/step)."""
    return int(round(periods * 3 * wavelength))


def config1() -> dict:
    """Homogeneous dielectric cylinder eps = 2, a = 10, 128^2, lambda = 40, 2000 steps."""
    return problem(nx=128, ny=128, radius=10.0, kind="homogeneous", eps1=2.0, wavelength=40.0, steps=2000)


def config2() -> dict:
    """Dielectric Janus eps1 = 2.25, eps2 = 4.0, phi0 = 30 deg, a = 64, 1024^2, lambda = 128, 20000 steps."""
    return problem(nx=1024, ny=1024, radius=64.0, kind="dielectric_janus", eps1=2.25, eps2=4.0, phi0_deg=30.0,
                   wavelength=128.0, steps=20000)


def config3(eps1: float = 2.0, phi0_deg: float = 0.0) -> dict:
    """Metallo-dielectric Janus, a = 48, 768^2, lambda = 96, 52 periods."""
    return problem(nx=768, ny=768, radius=48.0, kind="metallo_dielectric_janus", eps1=eps1, phi0_deg=phi0_deg,
                   wavelength=96.0, steps=steps_for(96.0))


def config3_sweep() -> list[dict]:
    return [config3(e, d) for e in (1.5, 2.0, 4.0, 8.0) for d in range(0, 181, 15)]


def config4_sweep(seed: int = 2509, eps1: float = 2.0) -> list[dict]:
    """Design map: eps2/eps1 in 16 log-spaced values 1.1..10 x 36 orientations.

    Radius a ~ U{32..128} per solve (seeded), grid 8a per side, lambda = 2a,
    52 periods, average the last 5.
    """
    rng = np.random.default_rng(seed)
    out = []
    ratios = [1.1 * (10.0 / 1.1) ** (i / 15.0) for i in range(16)]
    for i, r in enumerate(ratios):
        for j in range(36):
            a = int(rng.integers(32, 129))
            out.append(problem(nx=8 * a, ny=8 * a, radius=float(a), kind="dielectric_janus", eps1=eps1,
                               eps2=eps1 * r, phi0_deg=10.0 * j, wavelength=2.0 * a, steps=steps_for(2.0 * a)))
    return out


def config5_requests(seed: int = 22308, n_req: int = 256, rate: float = 20.0, a_min: int = 16, a_max: int = 256):
    """Serving: Poisson arrivals (mean `rate`/s) of dielectric Janus solves.

    a ~ U{a_min..a_max}, grid 8a, eps1, eps2 ~ U[1.5, 10], phi0 ~ U[0, 180) deg,
    lambda = 2a, 52 periods.  Returns [(arrival_seconds, problem), ...].
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_req):
        t += float(rng.exponential(1.0 / rate))
        a = int(rng.integers(a_min, a_max + 1))
        e1, e2 = (float(v) for v in rng.uniform(1.5, 10.0, size=2))
        phi = float(rng.uniform(0.0, 180.0))
        out.append((t, problem(nx=8 * a, ny=8 * a, radius=float(a), kind="dielectric_janus", eps1=e1, eps2=e2,
                               phi0_deg=phi, wavelength=2.0 * a, steps=steps_for(2.0 * a))))
    return out


def paper_mdjc_map(eps_stride: int = 1, phi_stride: int = 1) -> tuple[list[dict], list[float], list[float]]:
    """The metallo-dielectric design map of Sec. IV.A (Fig. HS75_Map): a / lambda = 1,
    a / dx = 40, domain L / a = 4 (160^2); phi0 = j pi / 90 (j = 0..180, i.e. 0..2 pi)
    and eps_r1 = 1 + 0.04 i (i = 0..100); 52 periods, the last 5 averaged.
    Returns (problems in row-major (eps, phi) order, eps axis, phi axis)."""
    a = 40
    eps = [round(1.0 + 0.04 * i, 10) for i in range(0, 101, eps_stride)]
    phi = [j * math.pi / 90 for j in range(0, 181, phi_stride)]
    probs = [problem(nx=4 * a, ny=4 * a, radius=float(a), kind="metallo_dielectric_janus", eps1=e, phi0=f,
                     wavelength=float(a), steps=steps_for(float(a))) for e in eps for f in phi]
    return probs, eps, phi


def paper_djc_map(eps1: float, eps_stride: int = 1, phi_stride: int = 1) -> tuple[list[dict], list[float], list[float]]:
    """A dielectric design map of Sec. IV.B (Fig. 2D_map; eps_r1 = 1, 2 or 5): a / lambda = 1,
    a / dx = 50, L / a = 4 (200^2); phi0 = j pi / 90 (j = 0..180) and
    eps_r2 / eps_r1 = 1 + 0.04 i (i = 0..100); 52 periods, the last 5 averaged.
    Returns (problems in row-major (ratio, phi) order, ratio axis, phi axis)."""
    a = 50
    ratio = [round(1.0 + 0.04 * i, 10) for i in range(0, 101, eps_stride)]
    phi = [j * math.pi / 90 for j in range(0, 181, phi_stride)]
    probs = [problem(nx=4 * a, ny=4 * a, radius=float(a), kind="dielectric_janus", eps1=float(eps1),
                     eps2=float(eps1) * r, phi0=f, wavelength=float(a), steps=steps_for(float(a)))
             for r in ratio for f in phi]
    return probs, ratio, phi


def paper_far_field_case(eps1: float, phi0: float, res: float = 50.0) -> dict:
    """The far-field validation of Sec. IV.A.1 (Fig. SW): metallo-dielectric
    Janus, a / lambda = 1, lambda_eps / dx = res (50 in the paper) inside the
    dielectric (lambda = res sqrt(eps_r1), rounded down so that 3 lambda is
    whole), L / a = 10; 52 periods."""
    lam = math.floor(3 * res * math.sqrt(eps1) + 1e-9) / 3
    n = int(math.ceil(10 * lam))
    return problem(nx=n, ny=n, radius=lam, kind="metallo_dielectric_janus", eps1=float(eps1), phi0=float(phi0),
                   wavelength=lam, steps=steps_for(lam))


def small_mdjc(eps1: float = 2.0, phi0_deg: float = 0.0, a: int = 16) -> dict:
    """Metallo-dielectric Janus at a / lambda = 0.5 on an 8a grid (oracle-sized)."""
    lam = 2.0 * a
    return problem(nx=8 * a, ny=8 * a, radius=float(a), kind="metallo_dielectric_janus", eps1=eps1,
                   phi0_deg=phi0_deg, wavelength=lam, steps=steps_for(lam))


def small_djc(eps1: float = 2.25, eps2: float = 4.0, phi0_deg: float = 30.0, a: int = 12, n: int | None = None,
              steps: int | None = None) -> dict:
    lam = 2.0 * a
    n = n or 8 * a
    return problem(nx=n, ny=n, radius=float(a), kind="dielectric_janus", eps1=eps1, eps2=eps2, phi0_deg=phi0_deg,
                   wavelength=lam, steps=steps or steps_for(lam, 20))


def random_small_problems(seed: int, count: int, a_min: int = 6, a_max: int = 20):
    """Mixed small problems (all three kinds, ragged grid sizes) for parity tests."""
    rng = np.random.default_rng(seed)
    kinds = ["homogeneous", "dielectric_janus", "metallo_dielectric_janus"]
    out = []
    for i in range(count):
        a = int(rng.integers(a_min, a_max + 1))
        lam = float(rng.choice([2 * a, 3 * a, 40]))
        lam = max(lam, 4.0 * math.sqrt(10.0))
        nx = int(2 * a + 2 * 3 + 10 + rng.integers(0, 40))
        ny = int(2 * a + 2 * 3 + 10 + rng.integers(0, 40))
        out.append(problem(nx=nx, ny=ny, radius=float(a), kind=kinds[i % 3], eps1=float(rng.uniform(1.5, 8.0)),
                           eps2=float(rng.uniform(1.5, 8.0)), phi0=float(rng.uniform(0, 2 * math.pi)),
                           wavelength=lam, steps=int(rng.integers(200, 700)), avg_periods=1))
    return out
