"""ctypes binding of the FP64 reference implementation (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU baseline leg
of the benchmark may import this module; the HIP library and its Python
binding never do.  Parameters are taken from any object that carries the
fields nx, ny, tau, G, G_ads1, G_ads2, tau_g, k_r, threshold, accel_x,
accel_y, x_in, x_out, y0, W; arrays are numpy, shape (ny, nx).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP over nodes)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double),
                ("G", C.c_double), ("G_ads", C.c_double * 2),
                ("tau_g", C.c_double), ("k_r", C.c_double),
                ("threshold", C.c_double), ("accel", C.c_double * 2),
                ("x_in", C.c_int32), ("x_out", C.c_int32), ("y0", C.c_int32),
                ("W", C.c_int32), ("c_eq", C.c_double), ("c_hold", C.c_double),
                ("hold_x", C.c_int32), ("solute_q", C.c_int32)]


class _Event(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("step", C.c_int64)]


class _Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double * 2),
                ("mass_removed", C.c_double * 2), ("solute", C.c_double),
                ("precipitate", C.c_double), ("solute_removed", C.c_double),
                ("front_z", C.c_double), ("delta_e", C.c_double),
                ("closure_step", C.c_int64), ("n_solid", C.c_int64),
                ("n_events", C.c_int64), ("nonfinite", C.c_int32),
                ("pad", C.c_int32), ("r_min", C.c_double), ("r_ave", C.c_double),
                ("r_h", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params), P, P, P, P]
        L.orc_create_state.restype = P
        L.orc_create_state.argtypes = [C.POINTER(_Params), P, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_clone.restype = P
        L.orc_clone.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int64]
        L.orc_fields.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_forces.argtypes = [P, P, P]
        L.orc_get_state.argtypes = [P, P, P, P]
        L.orc_events.restype = C.c_int64
        L.orc_events.argtypes = [P, P, C.c_int64]
        L.orc_step_count.restype = C.c_int64
        L.orc_step_count.argtypes = [P]
        L.orc_observe.argtypes = [P, C.POINTER(_Obs)]
        L.orc_override.restype = C.c_int
        L.orc_override.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_int32]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.orc_check_params.restype = C.c_int
        L.orc_check_params.argtypes = [C.POINTER(_Params)]
        _lib = L
    return _lib


def _params(p) -> _Params:
    return _Params(int(p.nx), int(p.ny), float(p.tau), float(p.G),
                   (C.c_double * 2)(float(p.G_ads1), float(p.G_ads2)),
                   float(p.tau_g), float(p.k_r), float(p.threshold),
                   (C.c_double * 2)(float(p.accel_x), float(p.accel_y)),
                   int(p.x_in), int(p.x_out), int(p.y0), int(p.W),
                   float(getattr(p, "c_eq", 0.0)), float(getattr(p, "c_hold", 0.0)),
                   int(getattr(p, "hold_x", 0)), int(getattr(p, "solute_q", 0)))


def _ptr(a):
    return None if a is None else a.ctypes.data


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, out.ctypes.data)
    return out


def params_valid(p) -> bool:
    pp = _params(p)
    return bool(lib().orc_check_params(C.byref(pp)))


EVENT_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("step", np.int64)])


class Oracle:
    """One FP64 simulation.  Build it from densities at rest (the initial
    condition of every workload) or from an arbitrary population state."""

    def __init__(self, p, solid, rho1=None, rho2=None, conc=None, *,
                 f=None, g=None, m=None):
        self.p = p
        self.nx, self.ny = int(p.nx), int(p.ny)
        self._keep = []
        pp = _params(p)
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        L = lib()
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64)
            g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
            m = None if m is None else np.ascontiguousarray(m, dtype=np.float64)
            h = L.orc_create_state(C.byref(pp), _ptr(solid), _ptr(f), _ptr(g), _ptr(m))
        else:
            rho1 = np.ascontiguousarray(rho1, dtype=np.float64)
            rho2 = np.ascontiguousarray(rho2, dtype=np.float64)
            conc = None if conc is None else np.ascontiguousarray(conc, dtype=np.float64)
            h = L.orc_create(C.byref(pp), _ptr(solid), _ptr(rho1), _ptr(rho2), _ptr(conc))
        if not h:
            raise ValueError("oracle rejected the parameters or the mask")
        self.h = h

    def clone(self) -> "Oracle":
        new = object.__new__(Oracle)
        new.p, new.nx, new.ny, new._keep = self.p, self.nx, self.ny, []
        h = lib().orc_clone(self.h)
        if not h:
            raise MemoryError("oracle clone failed")
        new.h = h
        return new

    @classmethod
    def from_problem(cls, prob):
        return cls(prob.params, prob.solid, prob.rho1, prob.rho2, prob.conc)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def step(self, n: int = 1):
        lib().orc_step(self.h, int(n))

    @property
    def steps(self) -> int:
        return int(lib().orc_step_count(self.h))

    def fields(self) -> dict:
        sh = (self.ny, self.nx)
        out = {k: np.zeros(sh) for k in ("rho1", "rho2", "ux", "uy", "conc", "m")}
        out["solid"] = np.zeros(sh, dtype=np.uint8)
        lib().orc_fields(self.h, *(out[k].ctypes.data for k in
                                   ("rho1", "rho2", "ux", "uy", "conc", "m", "solid")))
        return out

    def forces(self):
        Fx = np.zeros((2, self.ny, self.nx))
        Fy = np.zeros((2, self.ny, self.nx))
        lib().orc_forces(self.h, Fx.ctypes.data, Fy.ctypes.data)
        return Fx, Fy

    def state(self):
        f = np.zeros((18, self.ny, self.nx))
        g = np.zeros((5, self.ny, self.nx))
        m = np.zeros((self.ny, self.nx))
        lib().orc_get_state(self.h, f.ctypes.data, g.ctypes.data, m.ctypes.data)
        return f, g, m

    def observe(self) -> dict:
        o = _Obs()
        lib().orc_observe(self.h, C.byref(o))
        return {"step": o.step, "mass": (o.mass[0], o.mass[1]),
                "mass_removed": (o.mass_removed[0], o.mass_removed[1]),
                "solute": o.solute, "precipitate": o.precipitate,
                "solute_removed": o.solute_removed, "front_z": o.front_z,
                "delta_e": o.delta_e, "closure_step": o.closure_step,
                "n_solid": o.n_solid, "n_events": o.n_events,
                "nonfinite": o.nonfinite, "r_min": o.r_min, "r_ave": o.r_ave, "r_h": o.r_h}

    def events(self) -> np.ndarray:
        L = lib()
        n = L.orc_events(self.h, None, 0)
        buf = np.zeros(n, dtype=EVENT_DTYPE)
        if n:
            L.orc_events(self.h, buf.ctypes.data, n)
        return buf

    def override(self, x: int, y: int, step: int, decision: bool):
        if lib().orc_override(self.h, int(x), int(y), int(step), int(bool(decision))):
            raise ValueError("bad override")
