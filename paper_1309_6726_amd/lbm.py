"""Thin ctypes binding of the C ABI in include/lbm.h.

Argument marshalling only: every step of the lattice Boltzmann path runs in
the HIP library (liblbm.so).  PyTorch provides the device workspace and the
stream.  The binding refuses to run without the built library; there is no
fallback.
"""

from __future__ import annotations

import ctypes as C
import os
import struct

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
FIELDS = ("rho1", "rho2", "ux", "uy", "conc", "precip", "solid")
MAGIC = 0x4C424D5853494D31
BLOB_VERSION = 2
SCHEMES = {"auto": 0, "populations": 1, "moments": 2}

EXPORTS = ("lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_observe", "lbm_fields",
           "lbm_events", "lbm_save", "lbm_load", "lbm_set_tile", "lbm_get_tile",
           "lbm_autotune", "lbm_set_load_hint", "lbm_get_load_hint",
           "lbm_set_scheme", "lbm_destroy", "lbm_strerror", "lbm_last_error",
           "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_set_tile",
           "lbm_batch_get_tile", "lbm_batch_set_scheme", "lbm_batch_set_graph", "lbm_batch_step",
           "lbm_batch_record_fronts", "lbm_batch_fronts", "lbm_batch_observe",
           "lbm_batch_fields", "lbm_batch_events", "lbm_batch_autotune", "lbm_batch_destroy",
           "surr_workspace_bytes", "surr_init", "surr_set_params", "surr_get_params",
           "surr_set_loss_weights", "surr_set_data", "surr_train_epoch", "surr_gradients",
           "surr_predict", "surr_predict_noalloc", "surr_destroy")


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double),
                ("G", C.c_double), ("G_ads", C.c_double * 2), ("tau_g", C.c_double),
                ("k_r", C.c_double), ("threshold", C.c_double), ("accel", C.c_double * 2),
                ("x_in", C.c_int32), ("x_out", C.c_int32), ("y0", C.c_int32),
                ("W", C.c_int32), ("c_eq", C.c_double), ("c_hold", C.c_double),
                ("hold_x", C.c_int32), ("solute_q", C.c_int32)]

    @classmethod
    def of(cls, p) -> "Params":
        """From any object with the inputs.Params fields."""
        return cls(int(p.nx), int(p.ny), float(p.tau), float(p.G),
                   (C.c_double * 2)(float(p.G_ads1), float(p.G_ads2)), float(p.tau_g),
                   float(p.k_r), float(p.threshold),
                   (C.c_double * 2)(float(p.accel_x), float(p.accel_y)),
                   int(p.x_in), int(p.x_out), int(p.y0), int(p.W),
                   float(getattr(p, "c_eq", 0.0)), float(getattr(p, "c_hold", 0.0)),
                   int(getattr(p, "hold_x", 0)), int(getattr(p, "solute_q", 0)))


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double * 2),
                ("mass_removed", C.c_double * 2), ("solute", C.c_double),
                ("precipitate", C.c_double), ("solute_removed", C.c_double),
                ("front_z", C.c_double), ("delta_e", C.c_double),
                ("closure_step", C.c_int64), ("n_solid", C.c_int64),
                ("n_events", C.c_int64), ("nonfinite", C.c_int32), ("pad", C.c_int32),
                ("r_min", C.c_double), ("r_ave", C.c_double), ("r_h", C.c_double)]

    def as_dict(self) -> dict:
        return {"step": self.step, "mass": (self.mass[0], self.mass[1]),
                "mass_removed": (self.mass_removed[0], self.mass_removed[1]),
                "solute": self.solute, "precipitate": self.precipitate,
                "solute_removed": self.solute_removed, "front_z": self.front_z,
                "delta_e": self.delta_e, "closure_step": self.closure_step,
                "n_solid": self.n_solid, "n_events": self.n_events,
                "r_min": self.r_min, "r_ave": self.r_ave, "r_h": self.r_h,
                "nonfinite": self.nonfinite}


EVENT_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("step", np.int64)])

_lib = None


def lib():
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        sig = {
            "lbm_workspace_bytes": [C.POINTER(Params), C.POINTER(C.c_size_t)],
            "lbm_init": [C.POINTER(Params), P, P, P, P, P, P, C.c_size_t, C.POINTER(P)],
            "lbm_step": [P, C.c_int64],
            "lbm_observe": [P, C.POINTER(Obs)],
            "lbm_fields": [P, C.c_uint32, P],
            "lbm_events": [P, C.c_int64, P, C.c_int64, C.POINTER(C.c_int64)],
            "lbm_save": [P, P, C.c_size_t, C.POINTER(C.c_size_t)],
            "lbm_load": [P, P, C.c_size_t],
            "lbm_set_tile": [P, C.c_int32, C.c_int32],
            "lbm_set_load_hint": [P, C.c_int32],
            "lbm_get_load_hint": [P, C.POINTER(C.c_int32)],
            "lbm_set_scheme": [P, C.c_int32],
            "lbm_batch_set_scheme": [P, C.c_int32],
            "lbm_get_tile": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "lbm_autotune": [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_double)],
            "lbm_batch_workspace_bytes": [C.c_int32, P, C.c_int32, C.POINTER(C.c_size_t)],
            "lbm_batch_init": [C.c_int32, P, P, P, P, P, C.c_int32, P, P, C.c_size_t,
                               C.POINTER(P)],
            "lbm_batch_set_tile": [P, C.c_int32, C.c_int32],
            "lbm_batch_get_tile": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "lbm_batch_set_graph": [P, C.c_int32],
            "lbm_batch_step": [P, C.c_int64],
            "lbm_batch_record_fronts": [P, C.c_int32],
            "lbm_batch_fronts": [P, P],
            "lbm_batch_observe": [P, C.c_int32, C.POINTER(Obs)],
            "lbm_batch_fields": [P, C.c_int32, C.c_uint32, P],
            "lbm_batch_events": [P, C.c_int32, C.c_int64, P, C.c_int64, C.POINTER(C.c_int64)],
            "lbm_batch_autotune": [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double)],
            "surr_workspace_bytes": [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
            "surr_init": [P, P, C.c_int32, C.c_int32, P, P, C.c_size_t, C.POINTER(P)],
            "surr_set_params": [P, P],
            "surr_get_params": [P, P],
            "surr_set_loss_weights": [P, P],
            "surr_set_data": [P, P, P, P, C.c_int32],
            "surr_train_epoch": [P, P, C.c_int32, C.c_float, C.POINTER(C.c_double)],
            "surr_gradients": [P, P, P, C.c_int32, P, C.POINTER(C.c_double)],
            "surr_predict": [P, P, C.c_int32, P],
            "surr_predict_noalloc": [P, P, C.c_int32, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.lbm_destroy.argtypes = [P]
        L.lbm_destroy.restype = None
        L.lbm_batch_destroy.argtypes = [P]
        L.lbm_batch_destroy.restype = None
        L.surr_destroy.argtypes = [P]
        L.surr_destroy.restype = None
        L.lbm_strerror.argtypes = [C.c_int]
        L.lbm_strerror.restype = C.c_char_p
        L.lbm_last_error.argtypes = []
        L.lbm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(status: int):
    if status != LBM_OK:
        L = lib()
        raise LbmError(status, f"{L.lbm_strerror(status).decode()}: {L.lbm_last_error().decode()}")


def workspace_bytes(p) -> int:
    n = C.c_size_t(0)
    pp = Params.of(p)
    check(lib().lbm_workspace_bytes(C.byref(pp), C.byref(n)))
    return n.value


def _ptr(a):
    return None if a is None else a.ctypes.data


class Sim:
    """A simulation on one GPU.  `device` and `stream` are torch objects; the
    workspace is a torch uint8 tensor owned by this object."""

    def __init__(self, p, solid, rho1, rho2, conc=None, *, device="cuda:0", stream=None,
                 tile=None, scheme=None):
        import torch
        self.p = p
        self.nx, self.ny = int(p.nx), int(p.ny)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(p)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws = (base + 255) // 256 * 256
        self._nbytes = nbytes
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        rho1 = np.ascontiguousarray(rho1, dtype=np.float64)
        rho2 = np.ascontiguousarray(rho2, dtype=np.float64)
        conc = None if conc is None else np.ascontiguousarray(conc, dtype=np.float64)
        pp = Params.of(p)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lbm_init(C.byref(pp), _ptr(solid), _ptr(rho1), _ptr(rho2), _ptr(conc),
                                 C.c_void_p(self.stream.cuda_stream), C.c_void_p(self._ws),
                                 nbytes, C.byref(h)))
        self.h = h
        if tile is not None:
            self.set_tile(*tile)
        if scheme is not None:
            self.set_scheme(scheme)

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(prob.params, prob.solid, prob.rho1, prob.rho2, prob.conc, **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        check(lib().lbm_step(self.h, int(n)))

    def observe(self) -> dict:
        o = Obs()
        check(lib().lbm_observe(self.h, C.byref(o)))
        return o.as_dict()

    def fields(self, names=FIELDS) -> dict:
        mask = 0
        for n in names:
            mask |= 1 << FIELDS.index(n)
        sel = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        buf = np.zeros((len(sel), self.ny, self.nx))
        check(lib().lbm_fields(self.h, mask, buf.ctypes.data))
        return {n: buf[k] for k, n in enumerate(sel)}

    def events(self) -> np.ndarray:
        n = C.c_int64(0)
        check(lib().lbm_events(self.h, 0, None, 0, C.byref(n)))
        buf = np.zeros(n.value, dtype=EVENT_DTYPE)
        if n.value:
            check(lib().lbm_events(self.h, 0, buf.ctypes.data, n.value, C.byref(n)))
        return buf

    def save(self) -> bytes:
        n = C.c_size_t(0)
        check(lib().lbm_save(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib().lbm_save(self.h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        check(lib().lbm_load(self.h, blob, len(blob)))

    def set_tile(self, tx: int, sy: int):
        check(lib().lbm_set_tile(self.h, int(tx), int(sy)))

    def set_load_hint(self, nontemporal: int):
        """0: normal cache policy on the step's loads, 1: non-temporal."""
        check(lib().lbm_set_load_hint(self.h, int(nontemporal)))

    def load_hint(self) -> int:
        v = C.c_int32(0)
        check(lib().lbm_get_load_hint(self.h, C.byref(v)))
        return v.value

    def set_scheme(self, scheme: str):
        """'auto' (moments at tau = 1), 'populations' or 'moments'."""
        check(lib().lbm_set_scheme(self.h, SCHEMES[scheme]))

    def tile(self):
        a, b = C.c_int32(0), C.c_int32(0)
        check(lib().lbm_get_tile(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, steps: int = 20):
        a, b, ms = C.c_int32(0), C.c_int32(0), C.c_double(0)
        check(lib().lbm_autotune(self.h, int(steps), C.byref(a), C.byref(b), C.byref(ms)))
        return (a.value, b.value), ms.value

    # -- arbitrary states through the checkpoint format --------------------
    def load_state(self, f, solid, g=None, m=None, step: int = 0):
        """Load populations f [18, ny, nx] (and g [5, ny, nx], m) as FP32/FP64
        through a checkpoint blob.  Populations at solid nodes are ignored."""
        blob = make_blob(self.p, f, solid, g, m, step)
        self.load(blob)


def make_blob(p, f, solid, g=None, m=None, step: int = 0) -> bytes:
    """Checkpoint blob (layout in include/lbm.h) for an arbitrary state."""
    nx, ny = int(p.nx), int(p.ny)
    N = nx * ny
    solute = float(p.tau_g) > 0
    react = float(p.k_r) > 0
    flags = (1 if solute else 0) | (2 if react else 0)
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(N)
    parts = [struct.pack("<Q4iqq", MAGIC, nx, ny, flags, BLOB_VERSION, int(step), 0)]
    ff = np.where(solid.reshape(1, ny, nx) != 0, 0.0, np.asarray(f)).astype(np.float32)
    parts.append(ff.reshape(18 * N).tobytes())
    if solute:
        gg = np.zeros((5, ny, nx)) if g is None else np.asarray(g)
        gg = np.where(solid.reshape(1, ny, nx) != 0, 0.0, gg).astype(np.float32)
        parts.append(gg.reshape(5 * N).tobytes())
    parts.append(solid.tobytes())
    if react:
        mm = np.zeros(N) if m is None else np.asarray(m, dtype=np.float64).reshape(N)
        parts.append(mm.astype(np.float64).tobytes())
        parts.append(np.where(solid != 0, 0, -1).astype(np.int32).tobytes())
        parts.append(np.zeros(3 * N, dtype=np.float32).tobytes())
    return b"".join(parts)


class Batch:
    """Many lattices advanced together (one launch per step for all of them).
    `problems`: sequence of objects with params, solid, rho1, rho2, conc."""

    def __init__(self, problems, *, nslots=0, device="cuda:0", stream=None, tile=None,
                 graph_chunk=0, scheme=None):
        import torch
        self.n = len(problems)
        self.problems = list(problems)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nslots = int(nslots)
        PA = Params * self.n
        self._params = PA(*[Params.of(pr.params) for pr in problems])
        n = C.c_size_t(0)
        check(lib().lbm_batch_workspace_bytes(self.n, self._params, self.nslots, C.byref(n)))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        self._arrays = []

        def ptrs(get, dtype):
            arr = (C.c_void_p * self.n)()
            for i, pr in enumerate(problems):
                a = get(pr)
                if a is None:
                    arr[i] = None
                    continue
                a = np.ascontiguousarray(a, dtype=dtype)
                self._arrays.append(a)
                arr[i] = a.ctypes.data
            return arr

        solid = ptrs(lambda pr: pr.solid, np.uint8)
        r1 = ptrs(lambda pr: pr.rho1, np.float64)
        r2 = ptrs(lambda pr: pr.rho2, np.float64)
        conc = ptrs(lambda pr: pr.conc, np.float64)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lbm_batch_init(self.n, self._params, solid, r1, r2, conc, self.nslots,
                                       C.c_void_p(self.stream.cuda_stream), C.c_void_p(ws),
                                       n.value, C.byref(h)))
        self._arrays = []
        self.h = h
        if scheme is not None:
            self.set_scheme(scheme)
        if tile is not None:
            self.set_tile(*tile)
        if graph_chunk:
            self.set_graph(graph_chunk)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, tx, sy):
        check(lib().lbm_batch_set_tile(self.h, int(tx), int(sy)))

    def set_scheme(self, scheme: str):
        check(lib().lbm_batch_set_scheme(self.h, SCHEMES[scheme]))

    def tile(self):
        a, b = C.c_int32(0), C.c_int32(0)
        check(lib().lbm_batch_get_tile(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_graph(self, chunk):
        check(lib().lbm_batch_set_graph(self.h, int(chunk)))

    def step(self, n=1):
        check(lib().lbm_batch_step(self.h, int(n)))

    def record_fronts(self, slot):
        check(lib().lbm_batch_record_fronts(self.h, int(slot)))

    def fronts(self) -> np.ndarray:
        out = np.zeros((self.n, self.nslots))
        check(lib().lbm_batch_fronts(self.h, out.ctypes.data))
        return out

    def observe(self, i) -> dict:
        o = Obs()
        check(lib().lbm_batch_observe(self.h, int(i), C.byref(o)))
        return o.as_dict()

    def fields(self, i, names=FIELDS) -> dict:
        pr = self.problems[i]
        ny, nx = int(pr.params.ny), int(pr.params.nx)
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        sel = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        buf = np.zeros((len(sel), ny, nx))
        check(lib().lbm_batch_fields(self.h, int(i), mask, buf.ctypes.data))
        return {nm: buf[k] for k, nm in enumerate(sel)}

    def events(self, i) -> np.ndarray:
        n = C.c_int64(0)
        check(lib().lbm_batch_events(self.h, int(i), 0, None, 0, C.byref(n)))
        buf = np.zeros(n.value, dtype=EVENT_DTYPE)
        if n.value:
            check(lib().lbm_batch_events(self.h, int(i), 0, buf.ctypes.data, n.value, C.byref(n)))
        return buf

    def autotune(self, steps=5):
        a, b, ms = C.c_int32(0), C.c_int32(0), C.c_double(0)
        check(lib().lbm_batch_autotune(self.h, int(steps), C.byref(a), C.byref(b), C.byref(ms)))
        return (a.value, b.value), ms.value
