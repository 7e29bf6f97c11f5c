"""Python binding of libjlb, the gfx950 library for the Janus-cylinder
electromagnetic lattice Boltzmann solve (arXiv 2509.22308).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libjlb.so``.  The functions keep the C names of
``include/jlb.h``; PyTorch provides device memory (workspace, field arrays)
and the stream.  Importing this module never loads the library; the first
call does, and raises if it has not been built (``python
paper_2509_22308_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjlb.so")

JLB_OK = 0
ERRORS = {-1: "JLB_E_ARG", -2: "JLB_E_GEOMETRY", -3: "JLB_E_RESOLUTION", -4: "JLB_E_WINDOW", -5: "JLB_E_OOM",
          -6: "JLB_E_DEVICE", -7: "JLB_E_NONFINITE", -8: "JLB_E_ADMISSION", -9: "JLB_E_STATE"}
KINDS = {"homogeneous": 0, "dielectric_janus": 1, "metallo_dielectric_janus": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
JLB_F_ALLOW_UNDERRESOLVED = 1
JLB_F_NO_GRAPH = 2
JLB_F_CENTRE = 4
REQ_STATUS = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class jlb_problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("radius", ctypes.c_double), ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
        ("phi0", ctypes.c_double), ("wavelength", ctypes.c_double), ("e0", ctypes.c_double),
        ("steps", ctypes.c_int64), ("avg_periods", ctypes.c_int32), ("ramp_periods", ctypes.c_int32),
        ("contour_offset", ctypes.c_double), ("contour_points", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("plateau_tol", ctypes.c_double), ("polarization", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("cx", ctypes.c_double), ("cy", ctypes.c_double),
    ]


class jlb_result(ctypes.Structure):
    _fields_ = [
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("tz", ctypes.c_double),
        ("fx_raw", ctypes.c_double), ("fy_raw", ctypes.c_double), ("tz_raw", ctypes.c_double),
        ("loop_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
        ("steps_done", ctypes.c_int64), ("window_steps", ctypes.c_int64),
        ("contour_points", ctypes.c_int32), ("graph_used", ctypes.c_int32),
        ("bytes_per_step", ctypes.c_int64), ("state_passes", ctypes.c_int64), ("energy_final", ctypes.c_double),
        ("main_ms", ctypes.c_double), ("main_launches", ctypes.c_int64), ("main_kind", ctypes.c_int32),
        ("main_variant", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class JlbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = ctypes.POINTER
_vp = ctypes.c_void_p


def load():
    """Load libjlb.so (raises if it is missing: there is no fallback path).

    PyTorch ships its own HIP runtime under the same soname as the system
    one.  The library must bind to the runtime torch uses, so torch is
    imported and its runtime initialised before the library is opened;
    opened first, the library would pull in the system runtime and the
    process would hold two, neither of which can then serve both."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python paper_2509_22308_amd/build.py")
        import torch
        torch.cuda.is_available()
        lib = ctypes.CDLL(LIB_PATH)
        sig = {
            "jlb_version": ([], ctypes.c_int),
            "jlb_last_error": ([], ctypes.c_char_p),
            "jlb_validate": ([_P(jlb_problem)], ctypes.c_int),
            "jlb_workspace_size": ([_P(jlb_problem), _P(ctypes.c_size_t)], ctypes.c_int),
            "jlb_material_map": ([_P(jlb_problem), _vp], ctypes.c_int),
            "jlb_solve": ([_P(jlb_problem), _vp, ctypes.c_size_t, _P(jlb_result), _vp, _vp, _vp, _vp, _vp],
                          ctypes.c_int),
            "jlb_solve_force_trace": ([_P(jlb_problem), _vp, ctypes.c_size_t, _P(jlb_result), _vp, _vp], ctypes.c_int),
            "jlb_solve_far_field": ([_P(jlb_problem), _vp, ctypes.c_size_t, _P(jlb_result), ctypes.c_int32, _vp,
                                     _vp], ctypes.c_int),
            "jlb_solve_static": ([_P(jlb_problem), _P(jlb_result), _vp, _vp, _vp, _vp], ctypes.c_int),
            "jlb_trajectory": ([ctypes.c_int32, ctypes.c_double, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _vp], ctypes.c_int),
            "jlb_time_step_kernel": ([_P(jlb_problem), _vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                      _P(ctypes.c_double), _vp], ctypes.c_int),
            "jlb_autotune": ([_P(jlb_problem), _vp, ctypes.c_size_t, ctypes.c_int32, _P(ctypes.c_int32),
                              _P(ctypes.c_double), _vp], ctypes.c_int),
            "jlb_set_step_variant": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "jlb_get_step_variant": ([ctypes.c_int32, _P(ctypes.c_int32)], ctypes.c_int),
            "jlb_set_two_step_variant": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "jlb_get_two_step_variant": ([ctypes.c_int32, _P(ctypes.c_int32)], ctypes.c_int),
            "jlb_time_two_step_kernel": ([_P(jlb_problem), _vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                          _P(ctypes.c_double), _vp], ctypes.c_int),
            "jlb_set_multi_step_variant": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "jlb_get_multi_step_variant": ([ctypes.c_int32, _P(ctypes.c_int32)], ctypes.c_int),
            "jlb_multi_step_shape": ([ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32)], ctypes.c_int),
            "jlb_time_multi_step_kernel": ([_P(jlb_problem), _vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                            _P(ctypes.c_double), _vp], ctypes.c_int),
            "jlb_copy_bandwidth": ([ctypes.c_size_t, ctypes.c_int32, _P(ctypes.c_double), _vp], ctypes.c_int),
            "jlb_engine_create": ([ctypes.c_size_t, ctypes.c_int32, _vp, _P(_vp)], ctypes.c_int),
            "jlb_engine_submit": ([_vp, _P(jlb_problem), _P(ctypes.c_uint64)], ctypes.c_int),
            "jlb_engine_run": ([_vp, ctypes.c_int64, _P(ctypes.c_int32)], ctypes.c_int),
            "jlb_engine_poll": ([_vp, ctypes.c_uint64, _P(ctypes.c_int32), _P(jlb_result)], ctypes.c_int),
            "jlb_engine_cancel": ([_vp, ctypes.c_uint64], ctypes.c_int),
            "jlb_engine_stats": ([_vp, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32),
                                  _P(ctypes.c_size_t)], ctypes.c_int),
            "jlb_engine_destroy": ([_vp], ctypes.c_int),
            "jlb_engine_set_policy": ([_vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "jlb_engine_set_four_step": ([_vp, ctypes.c_int32], ctypes.c_int),
            "jlb_engine_four_step_choice": ([_vp, ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_double),
                                             _P(ctypes.c_int32)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != JLB_OK:
        raise JlbError(rc, load().jlb_last_error().decode())


POLARIZATIONS = {"tm": 0, "te": 1, 0: 0, 1: 1}


def make_problem(d: dict, precision: str | int | None = None, flags: int = 0) -> jlb_problem:
    """jlb_problem from a problem dict (keys as in the seeded workloads)."""
    kind = d.get("kind", "homogeneous")
    prec = precision if precision is not None else d.get("precision", "fp64")
    phi0 = d.get("phi0")
    if phi0 is None:
        phi0 = math.radians(d.get("phi0_deg", 0.0))
    return jlb_problem(
        nx=int(d["nx"]), ny=int(d.get("ny", d["nx"])), kind=KINDS[kind] if isinstance(kind, str) else int(kind),
        precision=PRECISIONS[prec] if isinstance(prec, str) else int(prec), radius=float(d["radius"]),
        eps1=float(d.get("eps1", 1.0)), eps2=float(d.get("eps2", 1.0)), phi0=float(phi0),
        wavelength=float(d["wavelength"]), e0=float(d.get("e0", 1.0)), steps=int(d["steps"]),
        avg_periods=int(d.get("avg_periods", 5)), ramp_periods=int(d.get("ramp_periods", 1)),
        contour_offset=float(d.get("contour_offset", 3.0)), contour_points=int(d.get("contour_points", 0)),
        flags=int(flags | d.get("flags", 0) | (JLB_F_CENTRE if "cx" in d or "cy" in d else 0)), plateau_tol=float(d.get("plateau_tol", 0.0)),
        polarization=POLARIZATIONS[d.get("polarization", "tm")],
        cx=float(d.get("cx", 0.0)), cy=float(d.get("cy", 0.0)),
    )


def jlb_version() -> int:
    return load().jlb_version()


def jlb_validate(prob: jlb_problem) -> int:
    """Return code of the library's problem check (0 = valid)."""
    return load().jlb_validate(ctypes.byref(prob))


def jlb_last_error() -> str:
    return load().jlb_last_error().decode()


def jlb_workspace_size(prob: jlb_problem) -> int:
    n = ctypes.c_size_t(0)
    _check(load().jlb_workspace_size(ctypes.byref(prob), ctypes.byref(n)))
    return n.value


def jlb_material_map(prob: jlb_problem) -> np.ndarray:
    out = np.zeros((prob.ny, prob.nx), dtype=np.uint8)
    _check(load().jlb_material_map(ctypes.byref(prob), out.ctypes.data_as(_vp)))
    return out


def _dptr(t):
    return None if t is None else _vp(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def jlb_solve(prob: jlb_problem, workspace=None, ez=None, hx=None, hy=None, energy=None, stream=None) -> jlb_result:
    """One solve; workspace/fields/energy are CUDA tensors (or None)."""
    res = jlb_result()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_solve(ctypes.byref(prob), _dptr(workspace), nbytes, ctypes.byref(res), _dptr(ez), _dptr(hx),
                            _dptr(hy), _dptr(energy), _stream(stream)))
    return res


def jlb_solve_force_trace(prob: jlb_problem, force, workspace=None, stream=None) -> jlb_result:
    """One solve plus the instantaneous (F~x, F~y, M~z) after every step into the
    CUDA float64 tensor force[steps][3] (see jlb_solve_force_trace in include/jlb.h)."""
    res = jlb_result()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_solve_force_trace(ctypes.byref(prob), _dptr(workspace), nbytes, ctypes.byref(res), _dptr(force),
                                        _stream(stream)))
    return res


def jlb_solve_far_field(prob: jlb_problem, n_angles: int, s2, workspace=None, stream=None) -> jlb_result:
    """One solve plus the far-field intensity at n_angles lab angles into the
    CUDA float64 tensor s2 (see jlb_solve_far_field in include/jlb.h)."""
    res = jlb_result()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_solve_far_field(ctypes.byref(prob), _dptr(workspace), nbytes, ctypes.byref(res), int(n_angles),
                                      _dptr(s2), _stream(stream)))
    return res


JLB_STATIC_SCRATCH_BYTES = 64 << 20


def jlb_solve_static(prob: jlb_problem, ez=None, hx=None, hy=None, stream=None) -> jlb_result:
    """The solve of jlb_solve on the library-held scratch (no device allocation
    by the library; fields are optional CUDA float64 tensors [ny][nx])."""
    res = jlb_result()
    _check(load().jlb_solve_static(ctypes.byref(prob), ctypes.byref(res), _dptr(ez), _dptr(hx), _dptr(hy),
                                   _stream(stream)))
    return res


def jlb_time_step_kernel(prob: jlb_problem, warmup: int, launches: int, workspace=None, stream=None) -> float:
    ms = ctypes.c_double(0.0)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_time_step_kernel(ctypes.byref(prob), _dptr(workspace), nbytes, int(warmup), int(launches),
                                       ctypes.byref(ms), _stream(stream)))
    return ms.value


STEP_VARIANTS = {0: "direct 64x4", 1: "2-wide tile 64x4", 2: "4-wide tile 64x4", 3: "2-wide tile 256x1",
                 4: "4-wide tile 256x1", 5: "2-wide tile 256x2", 6: "4-wide tile 256x2"}
FP64_STEP_VARIANTS = {0: "direct 64x4", 1: "direct 256x1", 2: "direct 256x2", 3: "2-node 64x4", 4: "2-node 256x1"}
FP64_TWO_STEP_VARIANTS = {0: "FP64 two-step H10 X4", 1: "FP64 two-step H12 X4", 2: "FP64 two-step H12 X4 W3",
                          3: "FP64 two-step H12 X4 LA2", 4: "FP64 two-step H6 X8", 5: "FP64 two-step H8 X8",
                          6: "FP64 two-step H8 X8 LA2", 7: "FP64 two-step H12 X8"}
TWO_STEP_VARIANTS = {0: "two-step V1 H8 X2", 1: "two-step V1 H16 X2", 2: "two-step V2 H8 X2",
                     3: "two-step V2 H16 X2", 4: "two-step V1 H8 X8", 5: "two-step V2 H16 X8",
                     6: "two-step V2 H32 X8", 7: "two-step V1 H8 X8 LA2", 8: "two-step V1 H4 X8 LA2",
                     9: "two-step V1 H16 X8 LA2"}
MULTI_STEP_VARIANTS = {0: "four-step H10 X4", 1: "four-step H12 X4", 2: "four-step H16 X4",
                       3: "three-step H10 X4", 4: "three-step H12 X4", 5: "four-step H12 X8",
                       6: "three-step H7 X4", 7: "three-step H8 X4"}


def variant_name(precision, best: int) -> str:
    """Name of a jlb_autotune winner (single-step index, or len(STEP_VARIANTS) + two-step index)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if prec == 0:
        if best >= len(FP64_STEP_VARIANTS):
            return FP64_TWO_STEP_VARIANTS.get(best - len(FP64_STEP_VARIANTS), str(best))
        return FP64_STEP_VARIANTS.get(best, str(best))
    if best >= len(STEP_VARIANTS):
        return TWO_STEP_VARIANTS.get(best - len(STEP_VARIANTS), str(best))
    return STEP_VARIANTS.get(best, str(best))


def jlb_autotune(prob: jlb_problem, launches: int = 20, workspace=None, stream=None):
    """Times every step variant of prob's precision (single steps, then
    two-step and multi-step kernels per lattice step); returns (best, [ms per
    step]); the multi-step choice is reported by jlb_get_multi_step_variant."""
    best = ctypes.c_int32(0)
    ms = (ctypes.c_double * (len(STEP_VARIANTS) + len(TWO_STEP_VARIANTS) + len(MULTI_STEP_VARIANTS)))()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_autotune(ctypes.byref(prob), _dptr(workspace), nbytes, int(launches), ctypes.byref(best), ms,
                               _stream(stream)))
    return best.value, list(ms)


def jlb_copy_bandwidth(nbytes: int, launches: int = 10, stream=None) -> float:
    """Mean ms of a plain device copy of nbytes (reference kernel)."""
    ms = ctypes.c_double(0.0)
    _check(load().jlb_copy_bandwidth(int(nbytes), int(launches), ctypes.byref(ms), _stream(stream)))
    return ms.value


def jlb_set_step_variant(precision: int, variant: int):
    _check(load().jlb_set_step_variant(int(precision), int(variant)))


def jlb_get_step_variant(precision: int) -> int:
    v = ctypes.c_int32(0)
    _check(load().jlb_get_step_variant(int(precision), ctypes.byref(v)))
    return v.value


def jlb_set_two_step_variant(precision: int, variant: int):
    _check(load().jlb_set_two_step_variant(int(precision), int(variant)))


def jlb_get_two_step_variant(precision: int) -> int:
    v = ctypes.c_int32(0)
    _check(load().jlb_get_two_step_variant(int(precision), ctypes.byref(v)))
    return v.value


def jlb_time_two_step_kernel(prob: jlb_problem, warmup: int, launches: int, workspace=None, stream=None) -> float:
    """Mean ms of one launch of the current two-step kernel (two lattice steps)."""
    ms = ctypes.c_double(0.0)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_time_two_step_kernel(ctypes.byref(prob), _dptr(workspace), nbytes, int(warmup), int(launches),
                                           ctypes.byref(ms), _stream(stream)))
    return ms.value


def jlb_set_multi_step_variant(precision: int, variant: int):
    _check(load().jlb_set_multi_step_variant(int(precision), int(variant)))


def jlb_get_multi_step_variant(precision: int) -> int:
    v = ctypes.c_int32(0)
    _check(load().jlb_get_multi_step_variant(int(precision), ctypes.byref(v)))
    return v.value


def jlb_multi_step_shape(variant: int):
    """(steps per launch, rows per wavefront) of a multi-step variant."""
    d, r = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().jlb_multi_step_shape(int(variant), ctypes.byref(d), ctypes.byref(r)))
    return d.value, r.value


def jlb_time_multi_step_kernel(prob: jlb_problem, warmup: int, launches: int, workspace=None, stream=None) -> float:
    """Mean ms of one launch of the current multi-step kernel (S lattice steps)."""
    ms = ctypes.c_double(0.0)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().jlb_time_multi_step_kernel(ctypes.byref(prob), _dptr(workspace), nbytes, int(warmup), int(launches),
                                             ctypes.byref(ms), _stream(stream)))
    return ms.value


def solve(d: dict, precision: str = "fp64", fields: bool = False, energy: bool = False, flags: int = 0,
          device: str = "cuda", far_angles: int = 0, force_trace: bool = False) -> dict:
    """Convenience wrapper: torch-allocated workspace and outputs; returns
    numpy arrays.  far_angles > 0 runs jlb_solve_far_field (key "s2"; not
    combinable with fields or energy)."""
    import torch
    prob = make_problem(d, precision, flags)
    ws = torch.empty(jlb_workspace_size(prob), dtype=torch.uint8, device=device)
    if force_trace:
        if fields or energy or far_angles:
            raise ValueError("force_trace does not combine with fields, energy or far_angles")
        ft = torch.zeros((prob.steps, 3), dtype=torch.float64, device=device)
        out = jlb_solve_force_trace(prob, ft, ws).as_dict()
        out["force_trace"] = ft.cpu().numpy()
        return out
    if far_angles > 0:
        if fields or energy:
            raise ValueError("far_angles does not combine with fields or energy")
        s2 = torch.empty(far_angles, dtype=torch.float64, device=device)
        out = jlb_solve_far_field(prob, far_angles, s2, ws).as_dict()
        out["s2"] = s2.cpu().numpy()
        return out
    f = [torch.empty((prob.ny, prob.nx), dtype=torch.float64, device=device) for _ in range(3)] if fields else [None] * 3
    en = torch.empty(prob.steps, dtype=torch.float64, device=device) if energy else None
    res = jlb_solve(prob, ws, *f, en)
    out = res.as_dict()
    if fields:
        out.update(ez=f[0].cpu().numpy(), hx=f[1].cpu().numpy(), hy=f[2].cpu().numpy())
    if energy:
        out["energy"] = en.cpu().numpy()
    return out


class Engine:
    """Batched solves resident on one device (see jlb_engine_* in include/jlb.h)."""

    def __init__(self, budget_bytes: int, max_slots: int, stream=None):
        self._h = _vp()
        s = None if stream is None else _vp(stream.cuda_stream)
        _check(load().jlb_engine_create(int(budget_bytes), int(max_slots), s, ctypes.byref(self._h)))

    def submit(self, prob: jlb_problem) -> int:
        t = ctypes.c_uint64(0)
        _check(load().jlb_engine_submit(self._h, ctypes.byref(prob), ctypes.byref(t)))
        return t.value

    def run(self, steps: int) -> int:
        a = ctypes.c_int32(0)
        _check(load().jlb_engine_run(self._h, int(steps), ctypes.byref(a)))
        return a.value

    def poll(self, ticket: int):
        st = ctypes.c_int32(0)
        res = jlb_result()
        _check(load().jlb_engine_poll(self._h, int(ticket), ctypes.byref(st), ctypes.byref(res)))
        return REQ_STATUS[st.value], res

    def cancel(self, ticket: int):
        _check(load().jlb_engine_cancel(self._h, int(ticket)))

    POLICIES = {"fifo": 0, "sjf": 1}

    def set_policy(self, policy: str = "fifo", max_slots: int = 0):
        """Admission order ("fifo" or "sjf": smallest work first) and, when > 0, a new slot count."""
        _check(load().jlb_engine_set_policy(self._h, self.POLICIES[policy], int(max_slots)))

    def set_four_step(self, on: bool):
        """Four-step rounds for the two-step solves (on by default)."""
        _check(load().jlb_engine_set_four_step(self._h, int(bool(on))))

    def four_step_choice(self, precision: str = "fp32") -> dict:
        """The four-step shape the engine runs for precision, the last timing's
        ms per batched launch of each candidate and the timings taken so far."""
        v, n = ctypes.c_int32(-1), ctypes.c_int32(0)
        ms = (ctypes.c_double * len(MULTI_STEP_VARIANTS))()
        _check(load().jlb_engine_four_step_choice(self._h, PRECISIONS[precision], ctypes.byref(v), ms, ctypes.byref(n)))
        return {"variant": MULTI_STEP_VARIANTS.get(v.value) if v.value >= 0 else None,
                "ms_per_launch": {MULTI_STEP_VARIANTS[k]: ms[k] for k in range(len(ms)) if ms[k] > 0.0},
                "tunings": n.value}

    def stats(self) -> dict:
        q, r, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        b = ctypes.c_size_t()
        _check(load().jlb_engine_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f), ctypes.byref(b)))
        return {"queued": q.value, "resident": r.value, "finished": f.value, "bytes_in_use": b.value}

    def close(self):
        if self._h:
            _check(load().jlb_engine_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
