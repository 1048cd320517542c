"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to the plain sequential FP64 reference in
``bd_oracle.cpp``.  Only the test-suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It never imports the GPU
library and the GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction, no fast-math)."""
    src = os.path.join(_HERE, "bd_oracle.cpp")
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, src])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    V = ctypes.c_void_p
    lib.orc_philox4x32_10.argtypes = [V, V, V]
    lib.orc_philox4x32_10.restype = None
    lib.orc_normals.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, V]
    lib.orc_normals.restype = None
    lib.orc_orient2.argtypes = [V, V, V]
    lib.orc_orient2.restype = ctypes.c_double
    lib.orc_incircle.argtypes = [V, V, V, V]
    lib.orc_incircle.restype = ctypes.c_double
    lib.orc_inverted_edge_flip.argtypes = [V, V, V, V]
    lib.orc_inverted_edge_flip.restype = ctypes.c_int
    lib.orc_point_in_closed_triangle.argtypes = [V, V, V, V]
    lib.orc_point_in_closed_triangle.restype = ctypes.c_int
    lib.orc_delaunay.argtypes = [ctypes.c_int, V, V, ctypes.c_int]
    lib.orc_delaunay.restype = ctypes.c_int
    lib.orc_forces.argtypes = [ctypes.c_int, V, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, V, ctypes.c_int, V]
    lib.orc_forces.restype = None
    lib.orc_force_tangent.argtypes = [ctypes.c_int, V, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, V, V, V]
    lib.orc_force_tangent.restype = None
    lib.orc_wall.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_wall.restype = ctypes.c_double
    lib.orc_overlap_round.argtypes = [ctypes.c_int, V, V, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, V]
    lib.orc_overlap_round.restype = ctypes.c_int64
    lib.orc_overlap_round_pairs.argtypes = lib.orc_overlap_round.argtypes
    lib.orc_overlap_round_pairs.restype = ctypes.c_int64
    lib.orc_sim_new.argtypes = [ctypes.c_int, V, V, V, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.orc_sim_new.restype = V
    lib.orc_sim_step.argtypes = [V, ctypes.c_int64]
    lib.orc_sim_step.restype = ctypes.c_int
    lib.orc_sim_last_rounds.argtypes = [V]
    lib.orc_sim_last_rounds.restype = ctypes.c_int
    lib.orc_sim_set_overlap_method.argtypes = [V, ctypes.c_int]
    lib.orc_sim_set_overlap_method.restype = None
    lib.orc_sim_set_max_halvings.argtypes = [V, ctypes.c_int]
    lib.orc_sim_set_max_halvings.restype = None
    lib.orc_sim_dt_halvings.argtypes = [V]
    lib.orc_sim_dt_halvings.restype = ctypes.c_int64
    lib.orc_bridge.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, V, V, V, V, V, V]
    lib.orc_bridge.restype = None
    lib.orc_sim_get.argtypes = [V, V, V, V, V]
    lib.orc_sim_get.restype = None
    lib.orc_sim_forces.argtypes = [V, V]
    lib.orc_sim_forces.restype = None
    lib.orc_sim_triangles.argtypes = [V, V, ctypes.c_int]
    lib.orc_sim_triangles.restype = ctypes.c_int
    lib.orc_frame.argtypes = [ctypes.c_double, ctypes.c_double, V, ctypes.c_int]
    lib.orc_frame.restype = ctypes.c_int
    lib.orc_sim_set_tangent.argtypes = [V, V, V]
    lib.orc_sim_set_tangent.restype = None
    lib.orc_sim_get_tangent.argtypes = [V, V]
    lib.orc_sim_get_tangent.restype = None
    lib.orc_sim_frame_count.argtypes = [V]
    lib.orc_sim_frame_count.restype = ctypes.c_int
    lib.orc_sim_free.argtypes = [V]
    lib.orc_sim_free.restype = None
    lib.orc_sim_set_periodic.argtypes = [V]
    lib.orc_sim_set_periodic.restype = ctypes.c_int
    lib.orc_forces_periodic.argtypes = [ctypes.c_int, V, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, V,
                                        ctypes.c_int, V]
    lib.orc_forces_periodic.restype = None
    lib.orc_torus_delaunay.argtypes = [ctypes.c_int, V, ctypes.c_double, V, ctypes.c_int]
    lib.orc_torus_delaunay.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data


def _pt(xy) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(2))


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normals(n: int, seed: int, step: int, stream: int) -> np.ndarray:
    """Unclamped Box-Muller pairs for particle ids 0..n-1: array (n, 2)."""
    lib = _load()
    out = np.zeros((n, 2), dtype=np.float64)
    lib.orc_normals(int(n), ctypes.c_uint64(seed), int(step), int(stream), _p(out))
    return out


def orient2(a, b, c) -> float:
    return _load().orc_orient2(_p(_pt(a)), _p(_pt(b)), _p(_pt(c)))


def incircle(a, b, c, d) -> float:
    return _load().orc_incircle(_p(_pt(a)), _p(_pt(b)), _p(_pt(c)), _p(_pt(d)))


def inverted_edge_flip(v1, v2, v3, v4) -> bool:
    args = [_pt(v) for v in (v1, v2, v3, v4)]
    return bool(_load().orc_inverted_edge_flip(*[_p(a) for a in args]))


def point_in_closed_triangle(v1, v2, v3, p) -> bool:
    args = [_pt(v) for v in (v1, v2, v3, p)]
    return bool(_load().orc_point_in_closed_triangle(*[_p(a) for a in args]))


def delaunay(xy: np.ndarray) -> np.ndarray:
    """Finite Delaunay triangles (CCW, rows of 3 vertex ids) of points xy (n, 2)."""
    lib = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    n = xy.shape[0]
    cap = max(2 * n, 4)
    out = np.zeros((cap, 3), dtype=np.int32)
    nt = lib.orc_delaunay(int(n), _p(xy), _p(out), int(cap))
    if nt < 0:
        raise RuntimeError(f"oracle delaunay failed ({nt})")
    return out[:nt].copy()


def frame(L: float, rmax: float) -> np.ndarray:
    """Fixed frame points outside the walls of [0, L]^2 (rows x, y)."""
    lib = _load()
    cap = int(4 * (math.ceil((L + 4 * rmax) / (2 * rmax)) + 4))
    out = np.zeros((cap, 2), dtype=np.float64)
    m = lib.orc_frame(float(L), float(rmax), _p(out), cap)
    if m < 0:
        raise RuntimeError("frame buffer too small")
    return out[:m].copy()


def delaunay_with_frame(xy: np.ndarray, L: float, rmax: float) -> np.ndarray:
    """Delaunay triangles of the disks plus the wall frame (frame ids follow the disks)."""
    pts = np.concatenate([np.asarray(xy, dtype=np.float64), frame(L, rmax)])
    return delaunay(pts)


def forces(xy, species, K, kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0, idx=None, period=0.0) -> np.ndarray:
    """Pair forces by brute force over all pairs (Sec. 2.2); period > 0: periodic box of that side with
    minimum-image separations (Sec. 2.1)."""
    lib = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    K = np.ascontiguousarray(K, dtype=np.float64)
    S = K.shape[0]
    n = xy.shape[0]
    kd = 0 if kind == "power" else 1
    if idx is None:
        out = np.zeros((n, 2), dtype=np.float64)
        lib.orc_forces_periodic(n, _p(xy), _p(sp), S, _p(K), kd, q, A, lam, cutoff, float(period), None, n,
                                _p(out))
    else:
        ix = np.ascontiguousarray(idx, dtype=np.int32)
        out = np.zeros((ix.size, 2), dtype=np.float64)
        lib.orc_forces_periodic(n, _p(xy), _p(sp), S, _p(K), kd, q, A, lam, cutoff, float(period), _p(ix),
                                int(ix.size), _p(out))
    return out


def torus_delaunay(xy: np.ndarray, L: float) -> np.ndarray:
    """Delaunay triangulation of the flat torus [0, L)^2 (periodic box, Sec. 2.1): 2n triangles of ids,
    counter-clockwise in the frame of their nearest images."""
    lib = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    n = xy.shape[0]
    out = np.zeros((2 * n + 4, 3), dtype=np.int32)
    nt = lib.orc_torus_delaunay(n, _p(xy), float(L), _p(out), out.shape[0])
    if nt < 0:
        raise RuntimeError("oracle torus triangulation failed")
    return out[:nt].copy()


def force_tangent(xy, species, K, txy, tK=None, kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0) -> np.ndarray:
    """Directional derivative of the pair forces along (txy, tK), the oracle's forward-mode rule."""
    lib = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    K = np.ascontiguousarray(K, dtype=np.float64)
    t = np.ascontiguousarray(txy, dtype=np.float64).reshape(-1, 2)
    tk = None if tK is None else np.ascontiguousarray(tK, dtype=np.float64)
    out = np.zeros_like(xy)
    lib.orc_force_tangent(xy.shape[0], _p(xy), _p(sp), K.shape[0], _p(K), 0 if kind == "power" else 1, q, A, lam,
                          cutoff, _p(t), None if tk is None else _p(tk), _p(out))
    return out


def bridge(W, Th, seed, step, level, index, h, D, Dr, clip=3.0):
    """Noise increments of the two halves of interval (level, index) of a step (length h, increments W (n, 2)
    and Th (n,)): the oracle's Brownian bridge.  Returns (WL, WR, ThL, ThR)."""
    lib = _load()
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1, 2)
    Th = np.ascontiguousarray(Th, dtype=np.float64)
    n = W.shape[0]
    WL, WR = np.zeros_like(W), np.zeros_like(W)
    ThL, ThR = np.zeros_like(Th), np.zeros_like(Th)
    lib.orc_bridge(n, ctypes.c_uint64(seed), int(step), int(level), int(index), float(h), float(D), float(Dr),
                   float(clip), _p(W), _p(Th), _p(WL), _p(WR), _p(ThL), _p(ThR))
    return WL, WR, ThL, ThR


def wall(c: float, r: float, L: float) -> float:
    return _load().orc_wall(c, r, L)


def overlap_round(xy: np.ndarray, radii, L: float, f: float = 1.0, cap_frac: float = 0.5, contact_tol: float = 1e-9):
    """One Jacobi round on the Delaunay edges of xy; returns (new_xy, n_overlapping_edges, cap_hits)."""
    lib = _load()
    out = np.ascontiguousarray(xy, dtype=np.float64).copy()
    rad = np.ascontiguousarray(radii, dtype=np.float64)
    hits = np.zeros(1, dtype=np.int64)
    cnt = lib.orc_overlap_round(out.shape[0], _p(out), _p(rad), L, f, cap_frac, contact_tol, _p(hits))
    if cnt < 0:
        raise RuntimeError("oracle triangulation failed")
    return out, int(cnt), int(hits[0])


def overlap_round_pairs(xy: np.ndarray, radii, L: float, f: float = 1.0, cap_frac: float = 0.5,
                        contact_tol: float = 1e-9):
    """One Jacobi round over every overlapping pair (no triangulation); returns (new_xy, n_pairs, cap_hits)."""
    lib = _load()
    out = np.ascontiguousarray(xy, dtype=np.float64).copy()
    rad = np.ascontiguousarray(radii, dtype=np.float64)
    hits = np.zeros(1, dtype=np.int64)
    cnt = lib.orc_overlap_round_pairs(out.shape[0], _p(out), _p(rad), L, f, cap_frac, contact_tol, _p(hits))
    return out, int(cnt), int(hits[0])


STAT_NAMES = ("steps", "overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits",
              "reversals", "noise_clamps")
# options of the GPU library that do not change what the step computes (force tiling, precision of the
# pair sums): the oracle ignores them when it is built from the same workload with them
GPU_ONLY = ("fp32", "force_chunk", "force_per_lane", "force_launch")


class OracleSim:
    """Sequential FP64 reference simulation (one handle per system)."""

    def __init__(self, xy, radii, species, theta, K, kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0,
                 L=100.0, D=1.0, dt=1e-4, v0=0.0, Dr=0.0, seed=0, step0=0, overlap_factor=1.0,
                 cap_frac=0.5, noise_clip=3.0, contact_tol=1e-9, max_overlap_rounds=10000, overlap="delaunay",
                 max_dt_halvings=0, periodic=False):
        lib = _load()
        self._lib = lib
        self.xy0 = np.ascontiguousarray(xy, dtype=np.float64)
        self.n = self.xy0.shape[0]
        self._rad = np.ascontiguousarray(radii, dtype=np.float64)
        self._sp = np.ascontiguousarray(species, dtype=np.int32)
        self._th = np.ascontiguousarray(theta if theta is not None else np.zeros(self.n), dtype=np.float64)
        self._K = np.ascontiguousarray(K, dtype=np.float64)
        S = self._K.shape[0]
        self._h = lib.orc_sim_new(self.n, _p(self.xy0), _p(self._rad), _p(self._sp), _p(self._th), S,
                                  _p(self._K), 0 if kind == "power" else 1, q, A, lam, cutoff, L, D, dt, v0, Dr,
                                  ctypes.c_uint64(seed), int(step0), overlap_factor, cap_frac, noise_clip,
                                  contact_tol, int(max_overlap_rounds))
        if not self._h:
            raise RuntimeError("oracle: initial triangulation failed")
        lib.orc_sim_set_overlap_method(self._h, {"delaunay": 0, "verlet": 1}[overlap])
        lib.orc_sim_set_max_halvings(self._h, int(max_dt_halvings))
        self.periodic = bool(periodic)
        if self.periodic and lib.orc_sim_set_periodic(self._h) != 0:
            raise RuntimeError("oracle: torus triangulation failed")

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(K=w.K, kind=w.kind, q=w.q, A=w.A, lam=w.lam, cutoff=w.cutoff, L=w.L, D=w.D, dt=w.dt,
                  v0=w.v0, Dr=w.Dr, seed=w.seed, step0=w.step0, overlap_factor=w.overlap_factor,
                  cap_frac=w.cap_frac, noise_clip=w.noise_clip, contact_tol=w.contact_tol,
                  max_overlap_rounds=w.max_overlap_rounds, overlap=w.overlap, max_dt_halvings=w.max_dt_halvings,
                  periodic=getattr(w, "periodic", False))
        kw.update({k: v for k, v in over.items() if k not in GPU_ONLY})
        return cls(w.xy, w.radii, w.species, w.theta, **kw)

    def step(self, nsteps: int = 1) -> int:
        rc = self._lib.orc_sim_step(self._h, int(nsteps))
        if rc != 0:
            raise RuntimeError(f"oracle step failed rc={rc}")
        return rc

    def last_rounds(self) -> int:
        return self._lib.orc_sim_last_rounds(self._h)

    def state(self):
        xy = np.zeros((self.n, 2), dtype=np.float64)
        th = np.zeros(self.n, dtype=np.float64)
        step = np.zeros(1, dtype=np.int64)
        st = np.zeros(7, dtype=np.int64)
        self._lib.orc_sim_get(self._h, _p(xy), _p(th), _p(step), _p(st))
        stats = dict(zip(STAT_NAMES, (int(v) for v in st)))
        stats["dt_halvings"] = int(self._lib.orc_sim_dt_halvings(self._h))
        return xy, th, int(step[0]), stats

    def forces(self) -> np.ndarray:
        out = np.zeros((self.n, 2), dtype=np.float64)
        self._lib.orc_sim_forces(self._h, _p(out))
        return out

    def set_tangent(self, txy, tK=None):
        """Carry forward-mode tangents from now on: txy (n, 2) for the positions, tK (S, S) for K."""
        self._txy = np.ascontiguousarray(txy, dtype=np.float64).reshape(-1, 2)
        self._tK = None if tK is None else np.ascontiguousarray(tK, dtype=np.float64)
        self._lib.orc_sim_set_tangent(self._h, _p(self._txy), None if self._tK is None else _p(self._tK))

    def tangent(self) -> np.ndarray:
        out = np.zeros((self.n, 2), dtype=np.float64)
        self._lib.orc_sim_get_tangent(self._h, _p(out))
        return out

    def triangles(self) -> np.ndarray:
        cap = 2 * (self.n + self._lib.orc_sim_frame_count(self._h)) + 4
        out = np.zeros((cap, 3), dtype=np.int32)
        nt = self._lib.orc_sim_triangles(self._h, _p(out), cap)
        return out[:nt].copy()

    def close(self):
        if self._h:
            self._lib.orc_sim_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
