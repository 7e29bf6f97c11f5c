"""Far field (arXiv 2509.22308, Sec. II.A, Eq. scattering intensity) on the
GPU, through the C ABI's jlb_solve_far_field, against the FP64 oracle.

Bars: FP64 within 1e-11 of the peak intensity at every angle (the phasor sums
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

TOL = {"fp64": 1e-11, "fp32": 1e-3, "bf16": 1e-2}


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


@pytest.mark.parametrize("variant", [0, 4, 5])
def test_far_field_after_two_step_kernels(jlb, refs, variant):
    """The window runs in two-step launches until the last period."""
    prec = jlb.PRECISIONS["fp32"]
    before = jlb.jlb_get_two_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, variant)
        _print_case(f"mdjc-fp32-two-step-{variant}", CASES["mdjc"], 72)
        g = jlb.solve(CASES["mdjc"], "fp32", far_angles=72)
        plain = jlb.solve(CASES["mdjc"], "fp32")
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
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
    assert np.abs(g["s2"] - ref["s2"]).max() <= 1e-11 * ref["s2"].max()


def test_single_angle_is_the_forward_intensity(jlb, refs):
    g = jlb.solve(CASES["config1"], "fp64", far_angles=1)
    ref = refs["config1"]["s2"][0]
    assert abs(g["s2"][0] - ref) <= 1e-11 * ref


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
