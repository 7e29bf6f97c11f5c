"""TE^z polarisation (Hz, Ex, Ey) on the GPU through the C ABI, against the
FP64 oracle's TE^z form (the polarisation arXiv 2509.22308 leaves for later
work, Sec. I, on the same lattice and update of Sec. III).

Bars as for TM^z: FP64 forces within 1e-12 and fields within 1e-12 of the
field scale; FP32 / BF16 forces within 1e-3 / 1e-2 of max(|F|, 0.05); far
field FP64 within 1e-12 of the peak.  The engine runs TE^z solves next to
TM^z ones (FP64 single steps and FP32 / BF16 two-step launches in one batch)
and returns what jlb_solve returns, bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from precision import force_bound

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


def _te(p):
    return dict(p, polarization="te")


CASES = {
    "config1": _te(W.config1()),
    "mdjc": _te(W.small_mdjc(4.0, 30.0, a=16)),
    "ragged-djc": _te(W.problem(nx=101, ny=77, radius=17.3, kind="dielectric_janus", eps1=3.0, eps2=1.5,
                                phi0_deg=225.0, wavelength=40.0, steps=2000)),
}


def _print_case(label, p):
    print(f"[case] TE {label}: {p['kind']} {p['nx']}x{p['ny']} a={p['radius']} lambda={p['wavelength']} "
          f"steps={p['steps']}", flush=True)


@pytest.fixture(scope="module")
def refs(oracle):
    return {k: oracle.solve(p, far_angles=72) for k, p in CASES.items()}


@pytest.mark.parametrize("case", list(CASES))
def test_te_fp64_matches_the_oracle(jlb, refs, case):
    p = CASES[case]
    _print_case(f"{case}-fp64", p)
    g = jlb.solve(p, "fp64", fields=True)
    r = refs[case]
    for q in ("fx", "fy", "tz"):
        assert abs(g[q] - r[q]) <= 1e-12 * max(1.0, abs(r[q])), (q, g[q], r[q])
    s = max(np.abs(r[f]).max() for f in ("ez", "hx", "hy"))
    for f in ("ez", "hx", "hy"):
        assert np.abs(g[f] - r[f]).max() <= 1e-12 * s, f


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_te_reduced_precision_forces_within_targets(jlb, refs, precision, case):
    p = CASES[case]
    _print_case(f"{case}-{precision}", p)
    g = jlb.solve(p, precision)
    r = refs[case]
    for q in ("fx", "fy", "tz"):
        assert abs(g[q] - r[q]) <= force_bound(precision, r[q]), (q, g[q], r[q])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_te_far_field_matches_the_oracle(jlb, refs, precision):
    p = CASES["mdjc"]
    _print_case(f"far-field-{precision}", p)
    g = jlb.solve(p, precision, far_angles=72)
    ref = refs["mdjc"]["s2"]
    err = np.abs(g["s2"] - ref).max() / ref.max()
    assert err <= (1e-12 if precision == "fp64" else 1e-3), err


def test_te_and_tm_share_an_engine(jlb):
    """TE^z and TM^z solves in one engine, FP32 / BF16 on the two- and
    four-step kernels and FP64 on its two-step kernel, in both polarisations:
    each result equals its own jlb_solve bit for bit."""
    probs = [CASES["config1"], W.config1(), CASES["ragged-djc"], W.small_mdjc(4.0, 30.0, a=16), CASES["mdjc"]]
    precs = ["fp32", "fp32", "bf16", "fp64", "fp64"]
    prec = jlb.PRECISIONS["fp32"]
    before = jlb.jlb_get_two_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, 4)
        eng = jlb.Engine(1 << 30, 16)
        tickets = [eng.submit(jlb.make_problem(p, pr)) for p, pr in zip(probs, precs)]
        while True:
            eng.run(512)
            st = eng.stats()
            if st["queued"] == 0 and st["resident"] == 0:
                break
        outs = [eng.poll(t) for t in tickets]
        eng.close()
        alone = [jlb.solve(p, pr) for p, pr in zip(probs, precs)]
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
    for (status, res), ref, p in zip(outs, alone, probs):
        assert status == "done"
        for q in ("fx", "fy", "tz"):
            assert getattr(res, q) == ref[q], (p.get("polarization", "tm"), q, getattr(res, q), ref[q])
