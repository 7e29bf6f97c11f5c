"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64: forces within 1e-12 relative (of max(1, |F|)) and fields within
1e-12 of the field scale, element by element.  FP32 / BF16 (deviation
storage): forces within 1e-3 / 1e-2 relative plus the absolute floors
1e-5 / 1e-4, and every field within 1e-3 / 1e-2 of the field scale
(tests/precision.py); each case's errors are printed.
"""
import math

import numpy as np
import pytest

import workloads as W
from precision import check, force_bound

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


def _field_scale(ref):
    return max(np.abs(ref["ez"]).max(), np.abs(ref["hx"]).max(), np.abs(ref["hy"]).max())


def _check_fp64(gpu, ref, label=""):
    for q in ("fx", "fy", "tz"):
        assert abs(gpu[q] - ref[q]) <= 1e-12 * max(1.0, abs(ref[q])), (label, q, gpu[q], ref[q])
    assert abs(gpu["energy_final"] - ref["energy_final"]) <= 1e-12 * ref["energy_final"], (label, "energy_final")
    s = _field_scale(ref)
    for f in ("ez", "hx", "hy"):
        err = np.abs(gpu[f] - ref[f]).max()
        assert err <= 1e-12 * s, (label, f, err, s)


def _print_case(label, prob):
    print(f"[case] {label}: {prob['kind']} {prob['nx']}x{prob['ny']} a={prob['radius']} "
          f"lambda={prob['wavelength']} steps={prob['steps']}", flush=True)


def test_fp64_config1_matches_oracle(jlb, oracle):
    p = W.config1()
    _print_case("config1", p)
    _check_fp64(jlb.solve(p, "fp64", fields=True), oracle.solve(p), "config1")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fp64_ragged_mixed_problems_match_oracle(jlb, oracle, seed):
    rng = np.random.default_rng(seed)
    kinds = ["homogeneous", "dielectric_janus", "metallo_dielectric_janus"]
    for k in range(3):
        a = float(rng.integers(6, 16))
        lam = float(rng.choice([2 * a, 30.0, 3 * a]))
        nx = int(2 * a + 2 * 3 + 10 + rng.integers(0, 70))
        ny = int(2 * a + 2 * 3 + 10 + rng.integers(0, 70))
        T = int(round(3 * lam))
        p = W.problem(nx=nx, ny=ny, radius=a, kind=kinds[k], eps1=float(rng.uniform(1.5, 6.0)),
                      eps2=float(rng.uniform(1.5, 6.0)), phi0=float(rng.uniform(0, 2 * math.pi)), wavelength=lam,
                      steps=3 * T + int(rng.integers(0, T)), avg_periods=1, flags=1)
        _print_case(f"seed{seed}-{k}", p)
        _check_fp64(jlb.solve(p, "fp64", fields=True), oracle.solve(p), f"seed{seed}-{k}")


@pytest.mark.parametrize("kind,deg", [("dielectric_janus", 45.0), ("metallo_dielectric_janus", 135.0),
                                      ("metallo_dielectric_janus", 270.0)])
def test_fp64_interface_ties_and_conductor_links(jlb, oracle, kind, deg):
    p = W.problem(nx=96, ny=90, radius=14.0, kind=kind, eps1=3.0, eps2=7.0, phi0_deg=deg, wavelength=30.0,
                  steps=1200, avg_periods=2)
    _print_case(f"{kind}-{deg}", p)
    _check_fp64(jlb.solve(p, "fp64", fields=True), oracle.solve(p), f"{kind}-{deg}")


def test_fp64_graph_replay_equals_direct_launches(jlb):
    p = W.problem(nx=128, ny=100, radius=12.0, kind="dielectric_janus", eps1=2.0, eps2=5.0, phi0_deg=20.0,
                  wavelength=24.0, steps=72 * 12 + 17, avg_periods=3)
    _print_case("graph-vs-eager", p)
    a = jlb.solve(p, "fp64", fields=True)
    b = jlb.solve(p, "fp64", fields=True, flags=jlb.JLB_F_NO_GRAPH)
    assert a["graph_used"] == 1 and b["graph_used"] == 0
    for q in ("fx", "fy", "tz"):
        assert a[q] == b[q]
    for f in ("ez", "hx", "hy"):
        assert np.array_equal(a[f], b[f])


def test_fp64_energy_trace_matches_oracle(jlb, oracle):
    p = W.problem(nx=80, ny=72, radius=10.0, kind="metallo_dielectric_janus", eps1=2.0, phi0_deg=60.0,
                  wavelength=24.0, steps=500, avg_periods=2)
    _print_case("energy", p)
    g = jlb.solve(p, "fp64", energy=True)
    r = oracle.solve(p, energy=True, fields=False)
    assert np.max(np.abs(g["energy"] - r["energy"])) <= 1e-12 * np.max(np.abs(r["energy"]))


def test_fp64_symmetric_bodies_have_zero_lift_and_torque_on_gpu(jlb):
    for kind, deg in (("homogeneous", 0.0), ("metallo_dielectric_janus", 90.0), ("dielectric_janus", 270.0)):
        p = W.problem(nx=96, ny=96, radius=14.0, kind=kind, eps1=2.0, eps2=4.0, phi0_deg=deg, wavelength=30.0,
                      steps=1500)
        r = jlb.solve(p, "fp64")
        assert r["fx"] > 0.1 and abs(r["fy"]) < 1e-13 and abs(r["tz"]) < 1e-13, (kind, deg, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_shortest_solve_matches_oracle(jlb, oracle, precision):
    """The fewest steps the checks accept: the ramp period, then the averaged
    period (no period before the window; the window is one captured chunk)."""
    p = W.problem(nx=128, ny=112, radius=14.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=60.0,
                  wavelength=40.0, steps=240, avg_periods=1)
    _print_case(f"shortest-{precision}", p)
    g = jlb.solve(p, precision, fields=True)
    r = oracle.solve(p)
    if precision == "fp64":
        _check_fp64(g, r, "shortest")
    else:
        check("shortest", precision, g, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_no_scatterer_feels_no_force_on_gpu(jlb, precision):
    """The degenerate body (eps = 1 everywhere): forces and torque vanish to
    each precision's absolute floor, in both polarisations."""
    for pol in ("tm", "te"):
        p = W.problem(nx=160, ny=160, radius=20.0, kind="homogeneous", eps1=1.0, wavelength=40.0,
                      steps=W.steps_for(40.0, 20), avg_periods=5, polarization=pol)
        r = jlb.solve(p, precision)
        for q in ("fx", "fy", "tz"):
            assert abs(r[q]) <= force_bound(precision, 0.0), (pol, precision, q, r[q])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("case", ["config1", "djc", "mdjc"])
def test_reduced_precision_forces_within_targets(jlb, oracle, precision, case):
    if case == "config1":
        p = W.config1()
    elif case == "djc":
        p = W.problem(nx=192, ny=192, radius=24.0, kind="dielectric_janus", eps1=2.25, eps2=4.0, phi0_deg=30.0,
                      wavelength=48.0, steps=W.steps_for(48.0, 20))
    else:
        p = W.small_mdjc(4.0, 30.0, a=24)
    _print_case(f"{case}-{precision}", p)
    g = jlb.solve(p, precision, fields=True)
    r = oracle.solve(p)
    check(case, precision, g, r)


def test_config2_cropped_fp64_matches_oracle(jlb, oracle):
    """Config 2's body and materials (DJC 2.25 / 4.0, 30 deg) on a 256^2 crop."""
    p = W.problem(nx=256, ny=256, radius=16.0, kind="dielectric_janus", eps1=2.25, eps2=4.0, phi0_deg=30.0,
                  wavelength=32.0, steps=2400)
    _print_case("config2-cropped", p)
    _check_fp64(jlb.solve(p, "fp64", fields=True), oracle.solve(p), "config2-cropped")


def test_config2_full_size_properties(jlb):
    """Config 2 at its full size (its oracle comparison is in
    test_gpu_fullsize.py): FP32 agrees with FP64 on the GPU within the FP32
    target, and the mirrored orientation (150 deg) gives (Fx, -Fy, -Mz)."""
    p = W.config2()
    _print_case("config2-full", p)
    d = jlb.solve(p, "fp64")
    f = jlb.solve(p, "fp32")
    for q in ("fx", "fy", "tz"):
        assert abs(f[q] - d[q]) <= force_bound("fp32", d[q]), (q, f[q], d[q])
    m = jlb.solve(dict(p, phi0=math.pi - p["phi0"]), "fp64")
    assert abs(m["fx"] - d["fx"]) < 1e-10 and abs(m["fy"] + d["fy"]) < 1e-10 and abs(m["tz"] + d["tz"]) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_step_kernel_variants_give_identical_results(jlb, precision):
    """Every thread-to-node mapping the autotuner may pick computes the same
    arithmetic: fields and forces agree bit for bit (ragged sizes, conductor
    links, all four edges).  Two- and multi-step launches are switched off,
    so every step runs on the variant under test."""
    prec = jlb.PRECISIONS[precision]
    before = jlb.jlb_get_step_variant(prec)
    two0 = jlb.jlb_get_two_step_variant(prec)
    multi0 = jlb.jlb_get_multi_step_variant(prec) if precision != "fp64" else -1
    cases = [W.problem(nx=203, ny=150, radius=20.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=110.0,
                       wavelength=40.0, steps=700, avg_periods=1),
             W.problem(nx=130, ny=171, radius=16.0, kind="dielectric_janus", eps1=2.0, eps2=6.0, phi0_deg=45.0,
                       wavelength=40.0, steps=650, avg_periods=1)]
    try:
        jlb.jlb_set_two_step_variant(prec, -1)
        if precision != "fp64":
            jlb.jlb_set_multi_step_variant(prec, -1)
        for p in cases:
            outs = []
            names = jlb.FP64_STEP_VARIANTS if precision == "fp64" else jlb.STEP_VARIANTS
            for v in range(len(names)):
                _print_case(f"{precision} step variant {v}", p)
                jlb.jlb_set_step_variant(prec, v)
                o = jlb.solve(p, precision, fields=True)
                assert (o["main_kind"], o["main_variant"]) == (1, v) and o["state_passes"] == p["steps"], v
                outs.append(o)
            for v, o in enumerate(outs[1:], 1):
                for q in ("fx", "fy", "tz", "energy_final"):
                    assert o[q] == outs[0][q], (v, q)
                for f in ("ez", "hx", "hy"):
                    assert np.array_equal(o[f], outs[0][f]), (v, f, np.abs(o[f] - outs[0][f]).max())
    finally:
        jlb.jlb_set_step_variant(prec, before)
        jlb.jlb_set_two_step_variant(prec, two0)
        if precision != "fp64":
            jlb.jlb_set_multi_step_variant(prec, multi0)


@pytest.mark.parametrize("polarization", ["tm", "te"])
def test_fp64_two_step_kernels_equal_single_steps(jlb, polarization):
    """FP64 two steps per launch (the graph-replayed periods before the
    window): every variant equals the single-step solve bit for bit, fields
    and forces (ragged strips and row segments, a conductor, all four edges,
    the companion row, a short top segment of four rows)."""
    two0 = jlb.jlb_get_two_step_variant(0)
    cases = [W.problem(nx=203, ny=150, radius=20.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=110.0,
                       wavelength=40.0, steps=840, avg_periods=1),
             W.problem(nx=130, ny=171, radius=16.0, kind="dielectric_janus", eps1=2.0, eps2=6.0, phi0_deg=45.0,
                       wavelength=40.0, steps=720, avg_periods=1),
             W.problem(nx=530, ny=97, radius=20.0, kind="metallo_dielectric_janus", eps1=4.0, phi0_deg=315.0,
                       wavelength=40.0, steps=720, avg_periods=1),
             W.problem(nx=64, ny=20, radius=3.0, kind="dielectric_janus", eps1=2.0, eps2=3.0, phi0_deg=60.0,
                       wavelength=40.0, steps=720, avg_periods=1, contour_offset=2.0),
             # near the smallest grids the checks accept: one strip spans the
             # grid, and a five-row segment reaches the top edge
             W.problem(nx=20, ny=17, radius=2.0, kind="metallo_dielectric_janus", eps1=2.0, phi0_deg=30.0,
                       wavelength=20.0, steps=240, avg_periods=1, contour_offset=1.6),
             W.problem(nx=17, ny=20, radius=2.0, kind="metallo_dielectric_janus", eps1=2.0, phi0_deg=200.0,
                       wavelength=20.0, steps=241, avg_periods=1, contour_offset=1.6)]
    cases = [dict(p, polarization=polarization) for p in cases]
    try:
        for p in cases:
            _print_case(f"fp64 two-step {polarization}", p)
            jlb.jlb_set_two_step_variant(0, -1)
            ref = jlb.solve(p, "fp64", fields=True)
            assert ref["state_passes"] == p["steps"] and ref["main_kind"] == 1
            for v in range(len(jlb.FP64_TWO_STEP_VARIANTS)):
                jlb.jlb_set_two_step_variant(0, v)
                o = jlb.solve(p, "fp64", fields=True)
                assert (o["main_kind"], o["main_variant"]) == (2, v) and o["state_passes"] < p["steps"], v
                for q in ("fx", "fy", "tz", "energy_final"):
                    assert o[q] == ref[q], (v, q, o[q], ref[q])
                for f in ("ez", "hx", "hy"):
                    assert np.array_equal(o[f], ref[f]), (v, f, np.abs(o[f] - ref[f]).max())
    finally:
        jlb.jlb_set_two_step_variant(0, two0)


@pytest.mark.parametrize("polarization", ["tm", "te"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_two_step_kernels_equal_single_steps(jlb, precision, polarization):
    """A two-step launch (temporal blocking) takes the state from n to n + 2
    with the single-step arithmetic and the intermediate deviations rounded
    to the storage type: solves that run their out-of-window periods on any
    two-step variant equal the single-step solve bit for bit, fields and
    forces (ragged strips and row segments, conductor links, all edges, the
    companion row), in both polarisations."""
    prec = jlb.PRECISIONS[precision]
    before, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    jlb.jlb_set_multi_step_variant(prec, -1)  # the two-step kernels outside the window too
    cases = [W.problem(nx=203, ny=150, radius=20.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=110.0,
                       wavelength=40.0, steps=700, avg_periods=1),
             W.problem(nx=130, ny=171, radius=16.0, kind="dielectric_janus", eps1=2.0, eps2=6.0, phi0_deg=45.0,
                       wavelength=40.0, steps=650, avg_periods=1),
             W.problem(nx=530, ny=97, radius=20.0, kind="dielectric_janus", eps1=4.0, eps2=1.5, phi0_deg=200.0,
                       wavelength=40.0, steps=700, avg_periods=1)]
    cases = [dict(p, polarization=polarization) for p in cases]
    try:
        for p in cases:
            _print_case(f"two-step {precision} {polarization}", p)
            jlb.jlb_set_two_step_variant(prec, -1)
            ref = jlb.solve(p, precision, fields=True)
            assert ref["state_passes"] == p["steps"]
            for v in range(len(jlb.TWO_STEP_VARIANTS)):
                jlb.jlb_set_two_step_variant(prec, v)
                o = jlb.solve(p, precision, fields=True)
                assert o["graph_used"] == 1 and o["state_passes"] < p["steps"], (v, o["state_passes"])
                for q in ("fx", "fy", "tz"):
                    assert o[q] == ref[q], (v, q, o[q], ref[q])
                for f in ("ez", "hx", "hy"):
                    assert np.array_equal(o[f], ref[f]), (v, f, np.abs(o[f] - ref[f]).max())
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
        jlb.jlb_set_multi_step_variant(prec, multi0)


@pytest.mark.parametrize("polarization", ["tm", "te"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_multi_step_kernels_equal_single_steps(jlb, precision, polarization):
    """Three or four levels in flight per sweep: solves that run on any
    multi-step variant (the window too, with the intermediate levels'
    contour fields) equal the single-step solve bit for bit, fields and
    forces, whatever the two-step choice; grids from ny = 20 (the shortest a
    four-step H16 segment allows) to wide ragged strips, conductor links,
    all edges, the companion row."""
    prec = jlb.PRECISIONS[precision]
    two0, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    cases = [W.problem(nx=203, ny=150, radius=20.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=110.0,
                       wavelength=40.0, steps=720, avg_periods=1),
             W.problem(nx=130, ny=171, radius=16.0, kind="dielectric_janus", eps1=2.0, eps2=6.0, phi0_deg=45.0,
                       wavelength=40.0, steps=720, avg_periods=1),
             W.problem(nx=530, ny=97, radius=20.0, kind="dielectric_janus", eps1=4.0, eps2=1.5, phi0_deg=200.0,
                       wavelength=40.0, steps=720, avg_periods=1),
             W.problem(nx=64, ny=20, radius=3.0, kind="dielectric_janus", eps1=2.0, eps2=3.0, phi0_deg=60.0,
                       wavelength=40.0, steps=720, avg_periods=1, contour_offset=2.0)]
    cases = [dict(p, polarization=polarization) for p in cases]
    try:
        for p in cases:
            _print_case(f"multi-step {precision} {polarization}", p)
            jlb.jlb_set_two_step_variant(prec, -1)
            jlb.jlb_set_multi_step_variant(prec, -1)
            ref = jlb.solve(p, precision, fields=True)
            assert ref["state_passes"] == p["steps"]
            for v in range(len(jlb.MULTI_STEP_VARIANTS)):
                for two in (-1, 4):
                    jlb.jlb_set_two_step_variant(prec, two)
                    jlb.jlb_set_multi_step_variant(prec, v)
                    o = jlb.solve(p, precision, fields=True)
                    assert o["graph_used"] == 1 and o["state_passes"] < p["steps"] * 0.6, (v, o["state_passes"])
                    depth, _ = jlb.jlb_multi_step_shape(v)
                    # ramp, the periods before the window and the window on multi-step launches
                    assert o["state_passes"] == 720 // depth, o["state_passes"]
                    for q in ("fx", "fy", "tz"):
                        assert o[q] == ref[q], (v, two, q, o[q], ref[q])
                    for f in ("ez", "hx", "hy"):
                        assert np.array_equal(o[f], ref[f]), (v, two, f, np.abs(o[f] - ref[f]).max())
    finally:
        jlb.jlb_set_two_step_variant(prec, two0)
        jlb.jlb_set_multi_step_variant(prec, multi0)


def test_multi_step_config2_matches_single_steps(jlb):
    """The headline workload: forces identical to single steps for every
    multi-step variant."""
    p = W.config2()
    prec = jlb.PRECISIONS["fp32"]
    two0, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, -1)
        jlb.jlb_set_multi_step_variant(prec, -1)
        ref = jlb.solve(p, "fp32")
        jlb.jlb_set_two_step_variant(prec, 4)
        for v in range(len(jlb.MULTI_STEP_VARIANTS)):
            jlb.jlb_set_multi_step_variant(prec, v)
            o = jlb.solve(p, "fp32")
            print(f"[multi-step] config2 variant {v}: loop {o['loop_ms']:.1f} ms, passes {o['state_passes']}, "
                  f"pre-window {o['main_ms']:.1f} ms in {o['main_launches']} launches", flush=True)
            for q in ("fx", "fy", "tz"):
                assert o[q] == ref[q], (v, q, o[q], ref[q])
            # 384 ramp steps, 46 periods of 384 steps before the 1920-step window
            depth, _ = jlb.jlb_multi_step_shape(v)
            assert (o["main_kind"], o["main_variant"], o["main_launches"]) == (3, v, 46 * 384 // depth)
            assert 0.0 < o["main_ms"] < o["loop_ms"]
    finally:
        jlb.jlb_set_two_step_variant(prec, two0)
        jlb.jlb_set_multi_step_variant(prec, multi0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_pre_window_stretch_is_reported_per_kernel(jlb, precision):
    """jlb_result names the kernel of the graph-replayed periods before the
    window and counts its launches: single steps, two-step or multi-step by
    what is selected; the forces do not depend on it."""
    prec = jlb.PRECISIONS[precision]
    two0, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    p = W.problem(nx=203, ny=150, radius=20.0, kind="dielectric_janus", eps1=2.0, eps2=6.0, phi0_deg=45.0,
                  wavelength=40.0, steps=1080, avg_periods=2)  # T 120: 120 ramp, 720 before the 240-step window
    out = {}
    try:
        for two, multi in ((-1, -1), (4, -1), (4, 0), (4, 3)):
            jlb.jlb_set_two_step_variant(prec, two)
            jlb.jlb_set_multi_step_variant(prec, multi)
            out[(two, multi)] = jlb.solve(p, precision)
    finally:
        jlb.jlb_set_two_step_variant(prec, two0)
        jlb.jlb_set_multi_step_variant(prec, multi0)
    expect = {(-1, -1): (1, 720), (4, -1): (2, 360), (4, 0): (3, 180), (4, 3): (3, 240)}
    for key, (kind, launches) in expect.items():
        o = out[key]
        assert (o["main_kind"], o["main_launches"]) == (kind, launches), (key, o["main_kind"], o["main_launches"])
        assert 0.0 < o["main_ms"] < o["loop_ms"]
        for q in ("fx", "fy", "tz"):
            assert o[q] == out[(-1, -1)][q], (key, q)


def test_four_step_choice_gives_way_to_three_steps_on_odd_chunks(jlb):
    """lambda = 50: a period of 150 steps, chunks of 300 = 4 (mod 8), so the
    default four-step variant gives way to three-step H10 X4 (100 launches per
    chunk); the result still equals single steps bit for bit."""
    p = W.problem(nx=120, ny=100, radius=12.0, kind="dielectric_janus", eps1=2.0, eps2=4.0, phi0_deg=30.0,
                  wavelength=50.0, steps=900, avg_periods=1)  # ramp 150, 2 chunks of 300, window 150
    prec = jlb.PRECISIONS["fp32"]
    two0, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, -1)
        jlb.jlb_set_multi_step_variant(prec, -1)
        ref = jlb.solve(p, "fp32", fields=True)
        jlb.jlb_set_two_step_variant(prec, 4)
        jlb.jlb_set_multi_step_variant(prec, 0)
        o = jlb.solve(p, "fp32", fields=True)
    finally:
        jlb.jlb_set_two_step_variant(prec, two0)
        jlb.jlb_set_multi_step_variant(prec, multi0)
    assert (o["main_kind"], o["main_variant"], o["main_launches"]) == (3, 3, 200)
    for q in ("fx", "fy", "tz"):
        assert o[q] == ref[q], q
    for f in ("ez", "hx", "hy"):
        assert np.array_equal(o[f], ref[f]), f


def test_two_step_config2_matches_single_steps(jlb):
    """The headline workload with the autotuner's choice: forces identical to
    single steps."""
    p = W.config2()
    prec = jlb.PRECISIONS["fp32"]
    before, multi0 = jlb.jlb_get_two_step_variant(prec), jlb.jlb_get_multi_step_variant(prec)
    try:
        jlb.jlb_set_multi_step_variant(prec, -1)
        jlb.jlb_set_two_step_variant(prec, -1)
        ref = jlb.solve(p, "fp32")
        for v in range(len(jlb.TWO_STEP_VARIANTS)):
            jlb.jlb_set_two_step_variant(prec, v)
            o = jlb.solve(p, "fp32")
            for q in ("fx", "fy", "tz"):
                assert o[q] == ref[q], (v, q, o[q], ref[q])
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
        jlb.jlb_set_multi_step_variant(prec, multi0)


def test_plateau_stop_matches_the_oracle(jlb, oracle):
    """The plateau stop (Sec. III, energy reaching a constant) decides the same
    check point on the GPU as in the oracle; FP64 forces then agree to 1e-12,
    and FP32 with two-step kernels stops at the same step within 1e-3."""
    p = dict(W.config1(), plateau_tol=1e-3)
    _print_case("plateau", p)
    ref = oracle.solve(p)
    assert ref["steps_done"] < p["steps"]
    g = jlb.solve(p, "fp64", fields=True)
    assert g["steps_done"] == ref["steps_done"]
    _check_fp64(g, ref, "plateau fp64")
    prec = jlb.PRECISIONS["fp32"]
    before = jlb.jlb_get_two_step_variant(prec)
    try:
        jlb.jlb_set_two_step_variant(prec, 4)
        f = jlb.solve(p, "fp32")
    finally:
        jlb.jlb_set_two_step_variant(prec, before)
    assert f["steps_done"] == ref["steps_done"]
    for q in ("fx", "fy", "tz"):
        assert abs(f[q] - ref[q]) <= force_bound("fp32", ref[q]), (q, f[q], ref[q])
