"""Instantaneous force trace and off-centre bodies on the GPU, through the C
ABI (jlb_solve_force_trace, JLB_F_CENTRE), against the FP64 oracle.

Bars: FP64 within 1e-12 of max(1, |F|) at every step; FP32 / BF16 within
1e-3 / 1e-2 of the trace's largest magnitude.  The trace's mean over the
averaging window equals the solve's forces (Sec. II.B: the stress is linear
in the averaged products).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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
    "mdjc": W.small_mdjc(4.0, 30.0, a=16),
    "mdjc-te": dict(W.small_mdjc(4.0, 30.0, a=16), polarization="te"),
    "djc-off-centre": dict(W.small_djc(2.25, 4.0, 30.0, a=12), cx=50.0, cy=41.5),
}


@pytest.fixture(scope="module")
def refs(oracle):
    return {k: oracle.solve(p, fields=False, force_trace=True) for k, p in CASES.items()}


def _print_case(label, p):
    print(f"[case] trace {label}: {p['kind']} {p['nx']}x{p['ny']} a={p['radius']} steps={p['steps']}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_force_trace_matches_the_oracle(jlb, refs, precision, case):
    p = CASES[case]
    _print_case(f"{case}-{precision}", p)
    g = jlb.solve(p, precision, force_trace=True)
    ref = refs[case]["force_trace"]
    err = np.abs(g["force_trace"] - ref).max()
    scale = max(1.0, np.abs(ref).max())
    tol = {"fp64": 1e-12, "fp32": 1e-3, "bf16": 1e-2}[precision]
    assert err <= tol * scale, (case, precision, err)
    if precision == "fp64":
        T = int(round(3 * p["wavelength"]))
        mean = g["force_trace"][-p["avg_periods"] * T:].mean(axis=0)
        np.testing.assert_allclose(mean, [g["fx"], g["fy"], g["tz"]], rtol=0, atol=1e-12)
    plain = jlb.solve(p, precision)
    for q in ("fx", "fy", "tz"):
        assert g[q] == plain[q], (q, g[q], plain[q])


def test_off_centre_fp64_fields_match_the_oracle(jlb, oracle):
    p = CASES["djc-off-centre"]
    _print_case("off-centre fields", p)
    g = jlb.solve(p, "fp64", fields=True)
    r = oracle.solve(p)
    for q in ("fx", "fy", "tz"):
        assert abs(g[q] - r[q]) <= 1e-12 * max(1.0, abs(r[q])), (q, g[q], r[q])
    s = max(np.abs(r[f]).max() for f in ("ez", "hx", "hy"))
    for f in ("ez", "hx", "hy"):
        assert np.abs(g[f] - r[f]).max() <= 1e-12 * s, f
