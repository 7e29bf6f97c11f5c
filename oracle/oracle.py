"""ctypes front end of the plain FP64 CPU oracle (``jlb_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.
It shares no code with the HIP library: parameters arrive as plain dicts (the
same dicts the seeded input generators hand to the HIP path) and are marshalled
into the oracle's own struct here.

The oracle computes, in IEEE FP64 with no FMA contraction, the EM lattice
Boltzmann solve of arXiv 2509.22308 Sec. III (Eqs. LBGK equation and
equilibrium distribution functions) and the time-averaged Maxwell-stress
contour integral of Sec. II.B (Eqs. stress tensor average, force, torque),
normalised by F0 = pi a eps0 E0^2 / 4 and M0 = 2 F0 a.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jlb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MAT_VACUUM, MAT_REGION2, MAT_REGION3, MAT_PEC = 0, 1, 2, 3
KINDS = {"homogeneous": 0, "dielectric_janus": 1, "metallo_dielectric_janus": 2}


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("radius", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
        ("kind", ctypes.c_int32),
        ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
        ("phi0", ctypes.c_double), ("wavelength", ctypes.c_double), ("e0", ctypes.c_double),
        ("steps", ctypes.c_int64),
        ("avg_periods", ctypes.c_int32), ("ramp_periods", ctypes.c_int32),
        ("contour_offset", ctypes.c_double), ("contour_points", ctypes.c_int32),
        ("boundary", ctypes.c_int32), ("literal", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("plateau_tol", ctypes.c_double), ("far_angles", ctypes.c_int32), ("polarization", ctypes.c_int32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("tz", ctypes.c_double),
        ("fx_raw", ctypes.c_double), ("fy_raw", ctypes.c_double), ("tz_raw", ctypes.c_double),
        ("energy_final", ctypes.c_double), ("window_steps", ctypes.c_int64),
        ("contour_points", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("steps_done", ctypes.c_int64),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, SRC, "-lm",
        ])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB)
        lib.orc_mask.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        lib.orc_mask.restype = ctypes.c_int
        lib.orc_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(_Result)]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_ntff.argtypes = ([ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_double] + [ctypes.c_void_p] * 6
                                 + [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_void_p])
        lib.orc_ntff.restype = None
        lib.orc_contour_points.argtypes = [ctypes.POINTER(_Params)]
        lib.orc_contour_points.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


POLARIZATIONS = {"tm": 0, "te": 1, 0: 0, 1: 1}


def _params(prob: dict, boundary: str = "open", literal: bool = False, threads: int | None = None) -> _Params:
    kind = prob.get("kind", "homogeneous")
    kind = KINDS[kind] if isinstance(kind, str) else int(kind)
    phi0 = prob.get("phi0", None)
    if phi0 is None:
        phi0 = math.radians(prob.get("phi0_deg", 0.0))
    if threads is None:
        threads = int(os.environ.get("JLB_ORACLE_THREADS", os.cpu_count() or 1))
    return _Params(
        nx=int(prob["nx"]), ny=int(prob["ny"]), radius=float(prob["radius"]),
        cx=float(prob.get("cx", math.nan)), cy=float(prob.get("cy", math.nan)),
        kind=kind, eps1=float(prob.get("eps1", 1.0)), eps2=float(prob.get("eps2", 1.0)),
        phi0=float(phi0), wavelength=float(prob["wavelength"]), e0=float(prob.get("e0", 1.0)),
        steps=int(prob["steps"]), avg_periods=int(prob.get("avg_periods", 5)),
        ramp_periods=int(prob.get("ramp_periods", 1)),
        contour_offset=float(prob.get("contour_offset", 3.0)),
        contour_points=int(prob.get("contour_points", 0)),
        boundary={"open": 0, "periodic": 1, "x_open_y_periodic": 2}[boundary], literal=int(bool(literal)), threads=int(threads),
        plateau_tol=float(prob.get("plateau_tol", 0.0)),
        polarization=POLARIZATIONS[prob.get("polarization", "tm")],
    )


def mask(prob: dict) -> np.ndarray:
    """Material id per node, [ny][nx] uint8 (0 vacuum, 1 region II, 2 region III, 3 PEC)."""
    p = _params(prob)
    out = np.zeros((p.ny, p.nx), dtype=np.uint8)
    rc = _load().orc_mask(ctypes.byref(p), _ptr(out))
    if rc != 0:
        raise ValueError("oracle mask failed: %d" % rc)
    return out


def contour_points(prob: dict) -> int:
    p = _params(prob)
    return _load().orc_contour_points(ctypes.byref(p))


def solve(prob: dict, *, literal: bool = False, boundary: str = "open", mat: np.ndarray | None = None,
          state: np.ndarray | None = None, fields: bool = True, energy: bool = False,
          accumulators: bool = False, threads: int | None = None, far_angles: int = 0,
          force_trace: bool = False) -> dict:
    """Run the oracle.  Returns forces, optional fields, energy trace, final
    state, and the far-field intensity at far_angles lab angles (key "s2")."""
    p = _params(prob, boundary=boundary, literal=literal, threads=threads)
    p.far_angles = int(far_angles)
    if far_angles > 0 and (boundary != "open" or p.avg_periods <= 0):
        raise ValueError("the far field needs open edges and an averaging window (its last period)")
    shape = (p.ny, p.nx)
    if mat is not None:
        mat = np.ascontiguousarray(mat, dtype=np.uint8)
        assert mat.shape == shape
    st = None
    if state is not None:
        st = np.ascontiguousarray(state, dtype=np.float64).copy()
        assert st.shape == ((2, 7, 3) if literal else (11,)) + shape
    ez = np.zeros(shape) if fields else None
    hx = np.zeros(shape) if fields else None
    hy = np.zeros(shape) if fields else None
    en = np.zeros(max(p.steps, 1)) if energy else None
    ncp = _load().orc_contour_points(ctypes.byref(p))
    acc = np.zeros((ncp, 4)) if accumulators else None
    s2 = np.zeros(far_angles) if far_angles > 0 else None
    nc = _load().orc_contour_points(ctypes.byref(p)) if far_angles > 0 else 0
    ph = np.zeros((nc, 12)) if far_angles > 0 else None
    ftr = np.zeros((p.steps, 3)) if force_trace else None
    res = _Result()
    rc = _load().orc_run(ctypes.byref(p), _ptr(mat), _ptr(st), _ptr(ez), _ptr(hx), _ptr(hy), _ptr(en),
                         _ptr(acc), _ptr(s2), _ptr(ph), _ptr(ftr), ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle run failed: %d" % rc)
    out = {k: getattr(res, k) for k in ("fx", "fy", "tz", "fx_raw", "fy_raw", "tz_raw", "energy_final",
                                         "window_steps", "contour_points", "steps_done")}
    if fields:
        out.update(ez=ez, hx=hx, hy=hy)
    if energy:
        out["energy"] = en[: p.steps]
    if accumulators:
        out["acc"] = acc
    if ftr is not None:
        out["force_trace"] = ftr
    if s2 is not None:
        out["s2"] = s2
        # complex phasors at the contour samples: total (Ez, Hx, Hy), then incident
        out["phasors"] = ph[:, 0::2] + 1j * ph[:, 1::2]
    if st is not None:
        out["state"] = st
    return out


def ntff(rx, ry, nx, ny, w: float, ez, hx, hy, k0: float, ei2: float, nphi: int) -> np.ndarray:
    """The oracle's near-to-far-field transform on given complex phasors."""
    arr = [np.ascontiguousarray(a, dtype=np.float64) for a in (rx, ry, nx, ny)]
    comp = []
    for f in (ez, hx, hy):
        f = np.asarray(f, dtype=np.complex128)
        comp += [np.ascontiguousarray(f.real), np.ascontiguousarray(f.imag)]
    out = np.zeros(nphi)
    _load().orc_ntff(ctypes.c_int(len(arr[0])), *[_ptr(a) for a in arr], ctypes.c_double(w), *[_ptr(a) for a in comp],
                     ctypes.c_double(k0), ctypes.c_double(ei2), ctypes.c_int(nphi), _ptr(out))
    return out
