"""FP64 CPU oracle of the constant-OPL vectorial ray march (test infrastructure).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is checked
against.  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library;
both sides only consume the same seeded inputs (``workloads.py``).

``build()`` compiles ``vrt_oracle.c`` with gcc (IEEE double, no FMA contraction,
OpenMP across rays) into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vrt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KINDS = {"homogeneous": 0, "linear": 1, "luneburg": 2, "fiber": 3, "gaussian": 4, "grid": 5,
         "spherical": 6, "n2p": 7, "zernike": 8}
BOUNDARIES = {"box": 0, "sphere": 1, "cylinder": 2}

EXITED, MISSED, TRUNCATED, NO_PLANE, INVALID_INPUT, REFLECTED_AT_ENTRY = range(6)
F_NEAR_CRITICAL, F_TANGENT, F_STRAIGHT, F_BOUNDARY_TIR, F_NEAR_TIE, F_NEAR_GRAZING = 1, 2, 4, 8, 16, 32
# the three windows ten times wider
F_NEAR_CRITICAL_WIDE, F_NEAR_TIE_WIDE, F_NEAR_GRAZING_WIDE = 64, 128, 256


def build(force=True):
    """Compile the oracle (gcc, -O2 -ffp-contract=off -fno-fast-math -fopenmp)."""
    global _lib
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


class _Medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_params", C.c_int32), ("params", C.POINTER(C.c_double)),
                ("grid", C.POINTER(C.c_float)), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("bkind", C.c_int32), ("glo", C.c_double * 3),
                ("ghi", C.c_double * 3), ("bparams", C.c_double * 6), ("n_amb", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("dL0", C.c_double), ("max_steps", C.c_int64), ("eps_tan", C.c_double),
                ("crit_rad", C.c_double), ("tie_eps", C.c_double), ("plane_z", C.c_double),
                ("has_plane", C.c_int32),
                ("pad", C.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB_PATH)
        dp, u32p, i64 = C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.c_int64
        lib.orc_trace.argtypes = [C.POINTER(_Medium), C.POINTER(_Params), i64, dp, dp, dp, dp,
                                  u32p, u32p, u32p, u32p, u32p, C.c_int]
        lib.orc_trace.restype = C.c_int
        lib.orc_trace_path.argtypes = [C.POINTER(_Medium), C.POINTER(_Params), dp, dp, dp, i64,
                                       C.POINTER(C.c_int64), dp, dp, u32p, u32p, u32p, u32p,
                                       u32p]
        lib.orc_trace_path.restype = C.c_int
        lib.orc_eval.argtypes = [C.POINTER(_Medium), i64, dp, dp, dp]
        lib.orc_eval.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class _MediumHandle:
    """Keeps the numpy buffers referenced by the C struct alive."""

    def __init__(self, medium):
        self.params = np.ascontiguousarray(medium.get("params", np.zeros(0)), dtype=np.float64)
        if self.params.size == 0:
            self.params = np.zeros(1)
        s = _Medium()
        s.kind = KINDS[medium["kind"]]
        s.n_params = int(self.params.size)
        s.params = _ptr(self.params, C.c_double)
        if medium["kind"] == "grid":
            self.grid = np.ascontiguousarray(medium["grid"], dtype=np.float32)
            s.grid = _ptr(self.grid, C.c_float)
            s.nz, s.ny, s.nx = self.grid.shape
            for a in range(3):
                s.glo[a] = float(medium["grid_lo"][a])
                s.ghi[a] = float(medium["grid_hi"][a])
        bnd = medium["boundary"]
        s.bkind = BOUNDARIES[bnd["kind"]]
        bp = np.asarray(bnd["params"], dtype=np.float64)
        for i, v in enumerate(bp):
            s.bparams[i] = float(v)
        s.n_amb = float(medium["n_amb"])
        self.s = s


def _params(p):
    q = _Params()
    q.dL0 = p["dL0"]
    q.max_steps = p["max_steps"]
    q.eps_tan = p.get("eps_tan", 0.0)
    q.crit_rad = p.get("crit_rad", 1e-6)
    q.tie_eps = p.get("tie_eps", 1e-7)
    z = p.get("exit_plane_z")
    q.has_plane = 0 if z is None else 1
    q.plane_z = 0.0 if z is None else float(z)
    return q


def trace(medium, rays, params, n_threads=0):
    """Trace rays (P0, d0) through the medium.  Returns a dict of numpy arrays:
    P, D (n,3) float64 exit state; status, steps, ntir, nbtir, flags (n,) uint32;
    plus 'seconds' (wall time of the C call) and 'threads'."""
    lib = _load()
    P0 = np.ascontiguousarray(rays[0], dtype=np.float64)
    d0 = np.ascontiguousarray(rays[1], dtype=np.float64)
    n = P0.shape[0]
    h = _MediumHandle(medium)
    q = _params(params)
    out = {k: np.zeros((n, 3)) for k in ("P", "D")}
    for k in ("status", "steps", "ntir", "nbtir", "flags"):
        out[k] = np.zeros(n, dtype=np.uint32)
    t0 = time.perf_counter()
    rc = lib.orc_trace(C.byref(h.s), C.byref(q), n, _ptr(P0, C.c_double), _ptr(d0, C.c_double),
                       _ptr(out["P"], C.c_double), _ptr(out["D"], C.c_double),
                       _ptr(out["status"], C.c_uint32), _ptr(out["steps"], C.c_uint32),
                       _ptr(out["ntir"], C.c_uint32), _ptr(out["nbtir"], C.c_uint32),
                       _ptr(out["flags"], C.c_uint32), int(n_threads))
    out["seconds"] = time.perf_counter() - t0
    out["threads"] = int(n_threads) if n_threads > 0 else os.cpu_count()
    if rc != 0:
        raise ValueError("oracle rejected the medium / parameters")
    return out


def trace_path(medium, P0, d0, params, cap=None):
    """Trace one ray and return (path (m,3), result dict)."""
    lib = _load()
    h = _MediumHandle(medium)
    q = _params(params)
    P0 = np.ascontiguousarray(P0, dtype=np.float64)
    d0 = np.ascontiguousarray(d0, dtype=np.float64)
    if cap is None:
        cap = int(params["max_steps"]) + 16
    path = np.zeros((cap, 3))
    npath = C.c_int64(0)
    oP, oD = np.zeros(3), np.zeros(3)
    u = [np.zeros(1, dtype=np.uint32) for _ in range(5)]
    rc = lib.orc_trace_path(C.byref(h.s), C.byref(q), _ptr(P0, C.c_double), _ptr(d0, C.c_double),
                            _ptr(path, C.c_double), cap, C.byref(npath), _ptr(oP, C.c_double),
                            _ptr(oD, C.c_double), *[_ptr(x, C.c_uint32) for x in u])
    if rc != 0:
        raise ValueError("oracle rejected the medium / parameters")
    m = min(npath.value, cap)
    res = {"P": oP, "D": oD, "status": int(u[0][0]), "steps": int(u[1][0]),
           "ntir": int(u[2][0]), "nbtir": int(u[3][0]), "flags": int(u[4][0]),
           "n_path": npath.value}
    return path[:m].copy(), res


def evaluate(medium, P):
    """n and grad n of the medium at points P (m,3)."""
    lib = _load()
    h = _MediumHandle(medium)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 3)
    n = np.zeros(P.shape[0])
    g = np.zeros_like(P)
    rc = lib.orc_eval(C.byref(h.s), P.shape[0], _ptr(P, C.c_double), _ptr(n, C.c_double),
                      _ptr(g, C.c_double))
    if rc != 0:
        raise ValueError("bad medium")
    return n, g
