"""Batched engine on the GPU: many solves resident and stepped together.

A solve's outcome may not depend on what else is resident: the engine's
result equals the single-solve result bit for bit, alone or in any mix, in
every precision.  Admission respects the byte budget, and cancelled or
oversized requests behave as documented.
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


def _mix():
    """Uneven solves: three kinds, ragged grids, different steps and periods."""
    return [
        W.problem(nx=96, ny=90, radius=12.0, kind="metallo_dielectric_janus", eps1=3.0, phi0_deg=40.0,
                  wavelength=30.0, steps=700, avg_periods=2),
        W.problem(nx=140, ny=128, radius=16.0, kind="dielectric_janus", eps1=2.0, eps2=5.0, phi0_deg=200.0,
                  wavelength=40.0, steps=900, avg_periods=2),
        W.problem(nx=72, ny=80, radius=9.0, kind="homogeneous", eps1=2.5, wavelength=24.0, steps=500,
                  avg_periods=3),
        W.problem(nx=200, ny=170, radius=20.0, kind="dielectric_janus", eps1=4.0, eps2=1.5, phi0_deg=75.0,
                  wavelength=40.0, steps=650, avg_periods=1),
        W.problem(nx=64, ny=64, radius=8.0, kind="metallo_dielectric_janus", eps1=1.5, phi0_deg=300.0,
                  wavelength=20.0, steps=420, avg_periods=2),
        # an odd step count: a two-step engine ends this solve with one step
        W.problem(nx=110, ny=77, radius=11.0, kind="dielectric_janus", eps1=6.0, eps2=2.0, phi0_deg=135.0,
                  wavelength=30.0, steps=541, avg_periods=2),
    ]


def _run_engine(jlb, probs, budget=8 << 30, slots=64, chunk=300, four=True):
    eng = jlb.Engine(budget, slots)
    eng.set_four_step(four)
    tickets = [eng.submit(p) for p in probs]
    out = {}
    for _ in range(10000):
        eng.run(chunk)
        st = eng.stats()
        if st["queued"] == 0 and st["resident"] == 0:
            break
    for t in tickets:
        status, res = eng.poll(t)
        assert status == "done", status
        out[t] = res.as_dict()
    eng.close()
    return [out[t] for t in tickets]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_engine_equals_single_solves_bit_for_bit(jlb, precision):
    probs = [jlb.make_problem(p, precision) for p in _mix()]
    single = [jlb.solve(p, precision) for p in _mix()]
    batched = _run_engine(jlb, probs)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "fx_raw", "fy_raw", "tz_raw"):
            assert s[q] == b[q], (precision, q, s[q], b[q])


def test_result_alone_equals_result_in_a_mix(jlb):
    target = _mix()[1]
    mixed_precisions = ["fp32", "bf16", "fp64", "fp32", "bf16"]
    alone = _run_engine(jlb, [jlb.make_problem(target, "fp32")])[0]
    others = [jlb.make_problem(p, pr) for p, pr in zip(_mix(), mixed_precisions)]
    mixed = _run_engine(jlb, others[:3] + [jlb.make_problem(target, "fp32")] + others[3:], chunk=97)
    b = mixed[3]
    for q in ("fx", "fy", "tz"):
        assert alone[q] == b[q]


def test_admission_under_a_small_budget_serialises_requests(jlb):
    probs = [jlb.make_problem(p, "fp32") for p in _mix()]
    sizes = [jlb.jlb_workspace_size(p) for p in probs]
    budget = int(max(sizes) * 1.5)  # the whole mix does not fit at once
    assert sum(sizes) > budget
    eng = jlb.Engine(budget, 16)
    tickets = [eng.submit(p) for p in probs]
    peak = 0
    for _ in range(10000):
        eng.run(200)
        st = eng.stats()
        assert st["bytes_in_use"] <= budget
        peak = max(peak, st["resident"])
        if st["queued"] == 0 and st["resident"] == 0:
            break
    assert all(eng.poll(t)[0] == "done" for t in tickets)
    assert eng.stats()["finished"] == len(probs)
    assert 1 <= peak < len(probs)
    eng.close()


def test_cancel_and_oversized_requests(jlb):
    probs = [jlb.make_problem(p, "bf16") for p in _mix()]
    eng = jlb.Engine(64 << 20, 2)
    with pytest.raises(jlb.JlbError) as ei:
        eng.submit(jlb.make_problem(W.config2(), "fp64"))  # ~400 MB > 64 MB
    assert ei.value.code == -8
    tickets = [eng.submit(p) for p in probs]
    eng.run(50)                     # two resident, the rest queued
    st = eng.stats()
    assert st["resident"] == 2 and st["queued"] == len(probs) - 2
    eng.cancel(tickets[0])          # running
    eng.cancel(tickets[-1])         # queued
    for _ in range(1000):
        eng.run(400)
        st = eng.stats()
        if st["queued"] == 0 and st["resident"] == 0:
            break
    assert eng.poll(tickets[0])[0] == "cancelled" and eng.poll(tickets[-1])[0] == "cancelled"
    assert all(eng.poll(t)[0] == "done" for t in tickets[1:-1])
    with pytest.raises(jlb.JlbError):
        eng.cancel(tickets[1])      # already finished
    eng.close()


@pytest.fixture
def two_step(jlb):
    """Selects a two-step variant for FP32 and BF16 for the test, then restores."""
    before = {p: jlb.jlb_get_two_step_variant(jlb.PRECISIONS[p]) for p in ("fp32", "bf16")}

    def select(v):
        for p in ("fp32", "bf16"):
            jlb.jlb_set_two_step_variant(jlb.PRECISIONS[p], v)
    yield select
    for p, v in before.items():
        jlb.jlb_set_two_step_variant(jlb.PRECISIONS[p], v)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("variant", [0, 4, 5])
def test_two_step_engine_equals_single_solves_bit_for_bit(jlb, two_step, precision, variant):
    """Batched two-step launches (every solve at its own step, ramp and window
    included, a final single step for an odd count) equal single solves."""
    two_step(-1)
    single = [jlb.solve(p, precision) for p in _mix()]
    two_step(variant)
    batched = _run_engine(jlb, [jlb.make_problem(p, precision) for p in _mix()], chunk=256)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "fx_raw", "fy_raw", "tz_raw"):
            assert s[q] == b[q], (precision, variant, q, s[q], b[q])


@pytest.mark.parametrize("chunk", [256, 130])
@pytest.mark.parametrize("variant", [0, 2, 4, 6])
def test_fp64_two_step_engine_equals_single_solves_bit_for_bit(jlb, variant, chunk):
    """Batched FP64 two-step launches (every solve at its own step, ramp and
    window included, both levels' field planes by level parity, a window
    start between the two levels of a launch, a final single step for an
    odd count) equal single-step solves: forces and final energy."""
    v0 = jlb.jlb_get_two_step_variant(0)
    try:
        jlb.jlb_set_two_step_variant(0, -1)
        single = [jlb.solve(p, "fp64") for p in _mix()]
        jlb.jlb_set_two_step_variant(0, variant)
        batched = _run_engine(jlb, [jlb.make_problem(p, "fp64") for p in _mix()], chunk=chunk)
    finally:
        jlb.jlb_set_two_step_variant(0, v0)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "fx_raw", "fy_raw", "tz_raw", "energy_final"):
            assert s[q] == b[q], (variant, chunk, q, s[q], b[q])


@pytest.mark.parametrize("four", [True, False])
@pytest.mark.parametrize("chunk", [256, 130])
def test_four_step_engine_equals_single_solves_bit_for_bit(jlb, two_step, four, chunk):
    """Rounds of four steps: a solve with at least four more levels to go
    takes the round's batched four-step launch, inside its averaging window
    too (the launch keeps the intermediate levels' contour fields); a solve
    with one to three levels left takes double steps; every solve runs at
    its own step.  The mix has window starts that are not multiples of four
    (steps 530 and 361), so four-step rounds straddle a window start.  A run
    of 130 steps ends on a lone double
    step in which the four-step solves wait.  A grid too short for the
    variant (ny = 19) stays on two-step launches.  Each result equals its
    single solve bit for bit, with the engine's four-step rounds on and off
    (and single solves on no multi-step kernels)."""
    prec = jlb.PRECISIONS["fp32"]
    multi0 = jlb.jlb_get_multi_step_variant(prec)
    probs = _mix() + [W.problem(nx=64, ny=19, radius=3.0, kind="dielectric_janus", eps1=2.0, eps2=3.0,
                                phi0_deg=60.0, wavelength=40.0, steps=720, avg_periods=1, contour_offset=2.0)]
    try:
        two_step(-1)
        jlb.jlb_set_multi_step_variant(prec, -1)
        single = [jlb.solve(p, "fp32") for p in probs]
        two_step(4)
        batched = _run_engine(jlb, [jlb.make_problem(p, "fp32") for p in probs], chunk=chunk, four=four)
    finally:
        jlb.jlb_set_multi_step_variant(prec, multi0)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "energy_final"):
            assert s[q] == b[q], (four, chunk, q, s[q], b[q])
        assert b["steps_done"] == s["steps_done"]


def test_engine_times_its_four_step_shape_on_the_mix(jlb, two_step):
    """The engine times each four-step shape's batched launch on the resident
    mix, runs the fastest, and still equals the single solves bit for bit."""
    prec = jlb.PRECISIONS["bf16"]
    multi0 = jlb.jlb_get_multi_step_variant(prec)
    probs = _mix()
    try:
        two_step(-1)
        jlb.jlb_set_multi_step_variant(prec, -1)
        single = [jlb.solve(p, "bf16") for p in probs]
        two_step(4)
        eng = jlb.Engine(8 << 30, 64)
        assert eng.four_step_choice("bf16")["tunings"] == 0
        tickets = [eng.submit(jlb.make_problem(p, "bf16")) for p in probs]
        eng.run(128)
        choice = eng.four_step_choice("bf16")
        for _ in range(1000):
            st = eng.stats()
            if st["queued"] == 0 and st["resident"] == 0:
                break
            eng.run(256)
        batched = [eng.poll(t)[1].as_dict() for t in tickets]
        eng.close()
    finally:
        jlb.jlb_set_multi_step_variant(prec, multi0)
    print(f"[engine] four-step choice {choice}", flush=True)
    times = choice["ms_per_launch"]
    assert choice["tunings"] >= 1
    assert sorted(times) == sorted(["four-step H10 X4", "four-step H12 X4", "four-step H16 X4", "four-step H12 X8"])
    assert all(t > 0.0 for t in times.values())
    assert choice["variant"] == min(times, key=times.get)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "energy_final"):
            assert s[q] == b[q], (q, s[q], b[q])


def test_two_step_and_single_step_solves_share_an_engine(jlb, two_step):
    """FP64 solves on single steps and FP32 / BF16 solves on two-step launches
    in one engine, admitted at different times: each equals its single solve."""
    two_step(5)
    precs = ["fp64", "fp32", "bf16", "fp32", "bf16", "fp64"]
    single = [jlb.solve(p, pr) for p, pr in zip(_mix(), precs)]
    batched = _run_engine(jlb, [jlb.make_problem(p, pr) for p, pr in zip(_mix(), precs)],
                          budget=sum(jlb.jlb_workspace_size(jlb.make_problem(p, pr)) for p, pr in
                                     zip(_mix()[:3], precs[:3])) + (1 << 24), chunk=128)
    for s, b in zip(single, batched):
        for q in ("fx", "fy", "tz", "energy_final"):
            assert s[q] == b[q], (q, s[q], b[q])


def test_smallest_work_first_admission(jlb):
    """With one slot and policy "sjf", queued requests run in order of work
    (cells x steps), whatever their arrival order; "fifo" keeps arrival
    order."""
    mix = _mix()
    work = [p["nx"] * p["ny"] * p["steps"] for p in mix]
    for policy in ("sjf", "fifo"):
        eng = jlb.Engine(8 << 30, 4)
        eng.set_policy(policy, 1)
        tickets = [eng.submit(jlb.make_problem(p, "fp32")) for p in mix]
        finished = []
        for _ in range(100000):
            eng.run(64)
            for k, t in enumerate(tickets):
                if k not in finished and eng.poll(t)[0] == "done":
                    finished.append(k)
            if len(finished) == len(mix):
                break
        eng.close()
        expect = sorted(range(len(mix)), key=lambda k: (work[k], k)) if policy == "sjf" else list(range(len(mix)))
        assert finished == expect, (policy, finished, expect)
    eng = jlb.Engine(1 << 30, 2)
    with pytest.raises(jlb.JlbError):
        eng.set_policy("fifo", -1)
    eng.close()


def test_a_failing_solve_does_not_stop_the_others(jlb):
    """Failure handling, forced from the host: a request whose fields
    overflow (a finite but huge amplitude, 1e200, in FP32) comes back with
    non-finite forces: a single solve returns JLB_E_NONFINITE, and in the
    engine the request ends "failed" while the rest of the mix finishes,
    each equal to its single solve."""
    probs = _mix()[:3]
    bad = dict(probs[1], e0=1e200)
    single = [jlb.solve(p, "fp32") for p in probs]
    with pytest.raises(jlb.JlbError) as err:
        jlb.solve(bad, "fp32")
    assert err.value.code == -7
    eng = jlb.Engine(8 << 30, 64)
    tickets = [eng.submit(jlb.make_problem(p, "fp32")) for p in probs]
    bad_ticket = eng.submit(jlb.make_problem(bad, "fp32"))
    for _ in range(1000):
        st = eng.stats()
        if st["queued"] == 0 and st["resident"] == 0:
            break
        eng.run(256)
    assert eng.poll(bad_ticket)[0] == "failed"
    for t, s in zip(tickets, single):
        status, res = eng.poll(t)
        assert status == "done"
        b = res.as_dict()
        for q in ("fx", "fy", "tz", "energy_final"):
            assert s[q] == b[q], (q, s[q], b[q])
    assert eng.stats()["finished"] == 4
    eng.close()


def test_an_empty_engine_runs_and_reports_nothing(jlb):
    eng = jlb.Engine(1 << 28, 4)
    assert eng.run(256) == 0
    assert eng.stats() == {"queued": 0, "resident": 0, "finished": 0, "bytes_in_use": 0}
    assert eng.four_step_choice("fp32")["tunings"] == 0
    eng.close()


def test_engine_rejects_the_plateau_stop(jlb):
    eng = jlb.Engine(1 << 30, 2)
    with pytest.raises(jlb.JlbError) as ei:
        eng.submit(jlb.make_problem(dict(_mix()[0], plateau_tol=1e-3), "fp32"))
    assert ei.value.code == -1
    eng.close()
