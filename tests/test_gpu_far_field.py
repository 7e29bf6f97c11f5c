"""Far field (arXiv 2509.22308, Sec. II.A, Eq. scattering intensity) on the
GPU, through the C ABI's jlb_solve_far_field, against the FP64 oracle.

Bars: FP64 within 1e-12 of the peak intensity at every angle (the phasor sums
are the oracle's up to summation order); FP32 / BF16 within 1e-3 / 1e-2 of
the peak.  The forces of a far-field solve equal those of jlb_solve bit for
bit (the last period runs as single steps, which equal the two-step kernels).
At the full 1024^2 size the far field is held to the momentum balance with
the contour stress, which holds at any size.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-3, "bf16": 1e-2}


@pytest.fixture(scope="module")
def jlb():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_22308_amd as J
    J.load()
    return J


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as O
    O.build(force=False)
    return O


CASES = {
    "config1": W.config1(),
    "mdjc": W.small_mdjc(4.0, 30.0, a=24),
    "ragged-djc": W.problem(nx=101, ny=77, radius=17.3, kind="dielectric_janus", eps1=3.0, eps2=1.5, phi0_deg=225.0,
                            wavelength=40.0, steps=2000),
}


def _print_case(label, prob, nphi):
    print(f"[case] far field {label}: {prob['kind']} {prob['nx']}x{prob['ny']} a={prob['radius']} "
          f"lambda={prob['wavelength']} steps={prob['steps']} angles={nphi}", flush=True)


@pytest.fixture(scope="module")
def refs(oracle):
    return {k: oracle.solve(p, fields=False, far_angles=72) for k, p in CASES.items()}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_far_field_matches_the_oracle(jlb, refs, precision, case):
    p = CASES[case]
    _print_case(f"{case}-{precision}", p, 72)
    g = jlb.solve(p, precision, far_angles=72)
    ref = refs[case]["s2"]
    err = np.abs(g["s2"] - ref).max() / ref.max()
    print(f"[far] {case} {precision}: max error / peak = {err:.3e}", flush=True)
    assert err <= TOL[precision], (case, precision, err)
    plain = jlb.solve(p, precision)
    for q in ("fx", "fy", "tz"):
        assert g[q] == plain[q], (q, g[q], plain[q])


def test_far_field_after_multi_step_kernels(jlb, refs):
    """The periods before the window and the window up to its last period on
    the four-step kernel (with the intermediate levels' contour fields), the
    last period on single steps."""
    prec = jlb.PRECISIONS["fp32"]
    before, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, 4)
        jlb.jlb_set_multi_step_variant(prec, 5)
        _print_case("mdjc-fp32-multi-step-5", CASES["mdjc"], 72)
        g = jlb.solve(CASES["mdjc"], "fp32", far_angles=72)
        plain = jlb.solve(CASES["mdjc"], "fp32")
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
        jlb.jlb_set_multi_step_variant(prec, multi0)
    ref = refs["mdjc"]["s2"]
    assert np.abs(g["s2"] - ref).max() <= 1e-3 * ref.max()
    assert plain["main_kind"] == 3 and plain["main_launches"] > 0
    for q in ("fx", "fy", "tz"):
        assert g[q] == plain[q]


@pytest.mark.parametrize("variant", [0, 4, 5])
def test_far_field_after_two_step_kernels(jlb, refs, variant):
    """The window runs in two-step launches until the last period (and, with
    the multi-step kernels off, the periods before it too)."""
    prec = jlb.PRECISIONS["fp32"]
    before, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    try:
        jlb.jlb_set_multi_step_variant(prec, -1)
        jlb.jlb_set_two_step_variant(prec, variant)
        _print_case(f"mdjc-fp32-two-step-{variant}", CASES["mdjc"], 72)
        g = jlb.solve(CASES["mdjc"], "fp32", far_angles=72)
        plain = jlb.solve(CASES["mdjc"], "fp32")
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
        jlb.jlb_set_multi_step_variant(prec, multi0)
    ref = refs["mdjc"]["s2"]
    assert np.abs(g["s2"] - ref).max() <= 1e-3 * ref.max()
    assert g["state_passes"] > plain["state_passes"] // 2  # the last period ran as single steps
    for q in ("fx", "fy", "tz"):
        assert g[q] == plain[q]


def test_far_field_with_the_plateau_stop(jlb, oracle):
    """The phasors cover the last period before the plateau stop."""
    p = dict(W.config1(), plateau_tol=1e-3)
    _print_case("plateau-fp64", p, 36)
    ref = oracle.solve(p, fields=False, far_angles=36)
    assert ref["steps_done"] < p["steps"]
    g = jlb.solve(p, "fp64", far_angles=36)
    assert g["steps_done"] == ref["steps_done"]
    assert np.abs(g["s2"] - ref["s2"]).max() <= 1e-12 * ref["s2"].max()


def test_single_angle_is_the_forward_intensity(jlb, refs):
    g = jlb.solve(CASES["config1"], "fp64", far_angles=1)
    ref = refs["config1"]["s2"][0]
    assert abs(g["s2"][0] - ref) <= 1e-12 * ref


def test_config2_full_size_far_field_momentum_balance(jlb):
    """1024^2, 20000 steps, FP32: drag and lift from the far field alone
    (lossless body, F = (1 / (2 k0)) int |S|^2 (x_hat - r_hat) dphi / F0)
    against the contour stress: within 3 % (lift: 0.01 + 3 %)."""
    p = W.config2()
    _print_case("config2-full-fp32", p, 720)
    g = jlb.solve(p, "fp32", far_angles=720)
    s2 = g["s2"]
    assert np.all(np.isfinite(s2)) and np.all(s2 >= 0.0)
    phi = 2 * math.pi * np.arange(720) / 720
    k0, f0 = 2 * math.pi / p["wavelength"], math.pi * p["radius"] / 4
    d = 2 * math.pi / 720
    fx = np.sum(s2 * (1 - np.cos(phi))) * d / (2 * k0 * f0)
    fy = -np.sum(s2 * np.sin(phi)) * d / (2 * k0 * f0)
    assert abs(fx - g["fx"]) < 0.03 * abs(g["fx"]), (fx, g["fx"])
    assert abs(fy - g["fy"]) < 0.01 + 0.03 * abs(g["fy"]), (fy, g["fy"])


def _fig_sw(jlb, eps1, phi0, res=50.0):
    from oracle import analytic as A
    p = W.paper_far_field_case(eps1, phi0, res)
    _print_case(f"fig-SW eps1={eps1} phi0={phi0:.4f} res={res}", p, 360)
    g = jlb.solve(p, "fp64", far_angles=360)
    x = 2 * math.pi
    C, S, _, _ = A.mdjc_coeffs(x, eps1, phi0, 1025)
    B, D = A.scattering_coeffs(C, S, x, phi0)
    phi = 2 * math.pi * np.arange(360) / 360
    ref = A.far_intensity(B, D, phi + phi0 + math.pi)
    rel = np.abs(g["s2"] - ref) / ref
    peak = np.abs(g["s2"] - ref).max() / ref.max()
    print(f"[far] fig-SW eps1={eps1} phi0={phi0:.4f} res={res}: median rel {np.median(rel):.4f}, "
          f"angles within 5 %: {np.mean(rel < 0.05):.2f}, max/peak {peak:.4f}", flush=True)
    return peak


# Largest error over the peak intensity each case is held to: about 1.5 times
# what it measures at lambda_eps / dx = 50, and never above the paper's 5 %
# (measured: 1.9 %, 0.8 % for eps_r1 = 1; 0.3 %, 0.7 % for 2; 2.2 %, 3.1 % for
# 5, at phi0 = 0 and -pi/4).
SW_BARS = {(1.0, 0.0): 0.03, (1.0, -math.pi / 4): 0.015, (2.0, 0.0): 0.01, (2.0, -math.pi / 4): 0.015,
           (5.0, 0.0): 0.035, (5.0, -math.pi / 4): 0.05}


@pytest.mark.parametrize("eps1", [1.0, 2.0, 5.0])
@pytest.mark.parametrize("phi0", [0.0, -math.pi / 4])
def test_far_field_reproduces_the_papers_validation(jlb, eps1, phi0):
    """Sec. IV.A.1 (Fig. SW): metallo-dielectric Janus, a = lambda, lambda_eps / dx
    = 50, L / a = 10, against the analytic scattered series (Eq. constants_Bm_Dm
    and the Hankel asymptotics).  The paper reports per-angle errors generally
    below 5 %; each case here is held to its own bar, all within 5 % of the
    peak intensity."""
    assert _fig_sw(jlb, eps1, phi0) < SW_BARS[(eps1, phi0)]


def test_far_field_error_with_resolution(jlb):
    """Refining lambda_eps / dx from 50 to 75 lowers the vacuum-half case's error
    (staircase and dispersion are discretisation errors), and the eps_r1 = 5,
    phi0 = -pi/4 case -- a conductor face on the lattice diagonal -- stays
    within the paper's 5 % at 50, 75 and 100 without growing."""
    e50 = _fig_sw(jlb, 1.0, 0.0, 50.0)
    e75 = _fig_sw(jlb, 1.0, 0.0, 75.0)
    assert e75 < 0.85 * e50
    d = [_fig_sw(jlb, 5.0, -math.pi / 4, r) for r in (50.0, 75.0, 100.0)]
    assert max(d) < 0.05 and d[2] <= d[0]
