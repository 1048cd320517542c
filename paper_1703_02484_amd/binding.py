"""ctypes binding of the C ABI in ``include/bd.h`` (argument marshalling only).

Every step of the simulation runs inside ``libbd.so``.  Loading fails loudly
when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbd.so")

BD_FORCE_POWER = 0
BD_FORCE_SCREENED = 1
BD_PREC_FP64 = 0
BD_PREC_FP32 = 1

EXPORTED = ("bd_strerror", "bd_last_error", "bd_params_default", "bd_init", "bd_step", "bd_forces",
            "bd_get_state", "bd_get_triangulation", "bd_get_frame", "bd_set_positions", "bd_set_stream",
            "bd_enable_kernel_timing", "bd_kernel_time", "bd_destroy")


class ForceParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("S", ctypes.c_int32), ("q", ctypes.c_double), ("A", ctypes.c_double),
                ("lam", ctypes.c_double), ("cutoff", ctypes.c_double), ("skin", ctypes.c_double),
                ("K", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("D", ctypes.c_double), ("dt", ctypes.c_double), ("v0", ctypes.c_double),
                ("Dr", ctypes.c_double), ("seed", ctypes.c_uint64), ("step0", ctypes.c_int64),
                ("overlap_factor", ctypes.c_double), ("cap_frac", ctypes.c_double),
                ("noise_clip", ctypes.c_double), ("contact_tol", ctypes.c_double),
                ("max_overlap_rounds", ctypes.c_int32),
                ("max_flip_rounds", ctypes.c_int32), ("force_precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


STAT_NAMES = ("steps", "overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits",
              "reversals", "noise_clamps", "flips_total", "inversion_flips", "flip_rounds_total", "kinetic_repairs",
              "host_rebuilds", "verlet_rebuilds")


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in STAT_NAMES] + [("reserved", ctypes.c_int64 * 3)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name in STAT_NAMES}


class BDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Loads libbd.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    V, P = ctypes.c_void_p, ctypes.POINTER
    lib.bd_strerror.argtypes = [ctypes.c_int]
    lib.bd_strerror.restype = ctypes.c_char_p
    lib.bd_last_error.argtypes = [V]
    lib.bd_last_error.restype = ctypes.c_char_p
    lib.bd_params_default.argtypes = [P(Params)]
    lib.bd_params_default.restype = None
    lib.bd_init.argtypes = [P(V), ctypes.c_int32, V, V, V, V, P(ForceParams), P(Params)]
    lib.bd_init.restype = ctypes.c_int
    lib.bd_step.argtypes = [V, ctypes.c_int64]
    lib.bd_step.restype = ctypes.c_int
    lib.bd_forces.argtypes = [V, V]
    lib.bd_forces.restype = ctypes.c_int
    lib.bd_get_state.argtypes = [V, V, V, P(ctypes.c_int64), P(Stats)]
    lib.bd_get_state.restype = ctypes.c_int
    lib.bd_get_triangulation.argtypes = [V, V, ctypes.c_int32, P(ctypes.c_int32)]
    lib.bd_get_triangulation.restype = ctypes.c_int
    lib.bd_get_frame.argtypes = [V, V, ctypes.c_int32, P(ctypes.c_int32)]
    lib.bd_get_frame.restype = ctypes.c_int
    lib.bd_set_positions.argtypes = [V, V]
    lib.bd_set_positions.restype = ctypes.c_int
    lib.bd_set_stream.argtypes = [V, V]
    lib.bd_set_stream.restype = ctypes.c_int
    lib.bd_enable_kernel_timing.argtypes = [V, ctypes.c_int]
    lib.bd_enable_kernel_timing.restype = ctypes.c_int
    lib.bd_kernel_time.argtypes = [V, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.bd_kernel_time.restype = ctypes.c_int
    lib.bd_destroy.argtypes = [V]
    lib.bd_destroy.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Sim:
    """One simulation handle (``bd_sim``) living on the current HIP device."""

    def __init__(self, xy, radii, species, theta, K, *, L, kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0,
                 skin=0.0, D=1.0, dt=1e-4, v0=0.0, Dr=0.0, seed=0, step0=0, overlap_factor=1.0, cap_frac=0.5,
                 noise_clip=3.0, contact_tol=1e-9, max_overlap_rounds=10000, max_flip_rounds=200, fp32=False):
        lib = load()
        self._lib = lib
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self.n = xy.shape[0]
        rad = np.ascontiguousarray(radii, dtype=np.float64)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        Km = np.ascontiguousarray(K, dtype=np.float64)
        fp = ForceParams(BD_FORCE_POWER if kind == "power" else BD_FORCE_SCREENED, Km.shape[0], q, A, lam, cutoff,
                         skin, _ptr(Km))
        p = Params()
        lib.bd_params_default(ctypes.byref(p))
        p.L, p.D, p.dt, p.v0, p.Dr = L, D, dt, v0, Dr
        p.seed, p.step0 = seed & (2**64 - 1), step0
        p.overlap_factor, p.cap_frac, p.noise_clip = overlap_factor, cap_frac, noise_clip
        p.contact_tol = contact_tol
        p.max_overlap_rounds, p.max_flip_rounds = max_overlap_rounds, max_flip_rounds
        p.force_precision = BD_PREC_FP32 if fp32 else BD_PREC_FP64
        h = ctypes.c_void_p()
        rc = lib.bd_init(ctypes.byref(h), self.n, _ptr(xy), _ptr(rad), _ptr(sp), None if th is None else _ptr(th),
                         ctypes.byref(fp), ctypes.byref(p))
        if rc != 0:
            raise BDError(rc, f"bd_init failed: {lib.bd_strerror(rc).decode()}")
        self._h = h

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(L=w.L, kind=w.kind, q=w.q, A=w.A, lam=w.lam, cutoff=w.cutoff, skin=w.skin, D=w.D, dt=w.dt,
                  v0=w.v0, Dr=w.Dr, seed=w.seed, step0=w.step0, overlap_factor=w.overlap_factor,
                  cap_frac=w.cap_frac, noise_clip=w.noise_clip, contact_tol=w.contact_tol,
                  max_overlap_rounds=w.max_overlap_rounds, fp32=w.fp32_forces)
        kw.update(over)
        return cls(w.xy, w.radii, w.species, w.theta, w.K, **kw)

    def _check(self, rc: int, what: str):
        if rc != 0:
            detail = self._lib.bd_last_error(self._h).decode()
            raise BDError(rc, f"{what} failed: {self._lib.bd_strerror(rc).decode()} ({detail})")

    def step(self, nsteps: int = 1):
        self._check(self._lib.bd_step(self._h, int(nsteps)), "bd_step")

    def forces(self) -> np.ndarray:
        out = np.zeros((self.n, 2), dtype=np.float64)
        self._check(self._lib.bd_forces(self._h, _ptr(out)), "bd_forces")
        return out

    def state(self):
        xy = np.zeros((self.n, 2), dtype=np.float64)
        th = np.zeros(self.n, dtype=np.float64)
        step = ctypes.c_int64()
        st = Stats()
        self._check(self._lib.bd_get_state(self._h, _ptr(xy), _ptr(th), ctypes.byref(step), ctypes.byref(st)),
                    "bd_get_state")
        return xy, th, int(step.value), st.as_dict()

    def frame(self) -> np.ndarray:
        m = ctypes.c_int32()
        self._check(self._lib.bd_get_frame(self._h, None, 0, ctypes.byref(m)), "bd_get_frame")
        out = np.zeros((m.value, 2), dtype=np.float64)
        self._check(self._lib.bd_get_frame(self._h, _ptr(out), m.value, ctypes.byref(m)), "bd_get_frame")
        return out

    def triangles(self) -> np.ndarray:
        m = ctypes.c_int32()
        self._check(self._lib.bd_get_frame(self._h, None, 0, ctypes.byref(m)), "bd_get_frame")
        cap = 2 * (self.n + m.value) + 4
        out = np.zeros((cap, 3), dtype=np.int32)
        nt = ctypes.c_int32()
        self._check(self._lib.bd_get_triangulation(self._h, _ptr(out), cap, ctypes.byref(nt)),
                    "bd_get_triangulation")
        return out[:nt.value].copy()

    def set_positions(self, xy):
        a = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self._check(self._lib.bd_set_positions(self._h, _ptr(a)), "bd_set_positions")

    def set_stream(self, stream_handle: Optional[int]):
        self._check(self._lib.bd_set_stream(self._h, stream_handle), "bd_set_stream")

    def enable_kernel_timing(self, on: bool = True):
        self._check(self._lib.bd_enable_kernel_timing(self._h, 1 if on else 0), "bd_enable_kernel_timing")

    def kernel_time(self):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self._lib.bd_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(cnt)), "bd_kernel_time")
        return float(ms.value), int(cnt.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
