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
BD_OVERLAP_DELAUNAY = 0
BD_OVERLAP_VERLET = 1

EXPORTED = ("bd_strerror", "bd_last_error", "bd_params_default", "bd_init", "bd_batch_init", "bd_batch_layout",
            "bd_get_force_config", "bd_step", "bd_forces", "bd_get_state", "bd_get_triangulation", "bd_get_frame",
            "bd_set_positions", "bd_set_graph_mode", "bd_set_tail_mode", "bd_set_stream", "bd_enable_kernel_timing", "bd_kernel_time",
            "bd_adjoint_begin", "bd_adjoint_backward", "bd_adjoint_backward_dev", "bd_get_state_dev",
            "bd_set_allocator", "bd_destroy", "bd_batch_step", "bd_batch_get_state", "bd_batch_destroy",
            "bd_rollout", "bd_backward", "bd_backward_dev", "bd_pair_forces_dev",
            "bd_pair_forces_dev_noalloc")


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
                ("force_chunk", ctypes.c_int32), ("force_per_lane", ctypes.c_int32),
                ("force_launch", ctypes.c_int32), ("overlap_method", ctypes.c_int32),
                ("max_dt_halvings", ctypes.c_int32), ("periodic", ctypes.c_int32)]


class ForceConfig(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("per_lane", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("grid", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("tuned_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


STAT_NAMES = ("steps", "overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits",
              "reversals", "noise_clamps", "flips_total", "inversion_flips", "flip_rounds_total", "kinetic_repairs",
              "host_rebuilds", "verlet_rebuilds", "host_continued", "dt_halvings")


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in STAT_NAMES] + [("reserved", ctypes.c_int64)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name in STAT_NAMES}


class BDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_lib = None
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = []   # every installed callback pair stays alive: handles keep the allocator they started with


def use_torch_allocator(enable: bool = True):
    """Device memory of handles created from now on comes from torch's caching allocator (or hipMalloc again)."""
    lib = load()
    if not enable:
        lib.bd_set_allocator(_ALLOC_FN(), _FREE_FN(), None)
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:   # out of memory: the library reports BD_ERR_OOM
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _allocator_refs.append(refs)
    rc = lib.bd_set_allocator(refs[0], refs[1], None)
    if rc != 0:
        raise BDError(rc, "bd_set_allocator failed")


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
    lib.bd_batch_init.argtypes = [P(V), ctypes.c_int32, V, V, V, V, V, V, V, P(ForceParams), P(Params)]
    lib.bd_batch_init.restype = ctypes.c_int
    lib.bd_batch_layout.argtypes = [V, P(ctypes.c_int32), V, V]
    lib.bd_batch_layout.restype = ctypes.c_int
    lib.bd_get_force_config.argtypes = [V, P(ForceConfig)]
    lib.bd_get_force_config.restype = ctypes.c_int
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
    lib.bd_set_tail_mode.argtypes = [V, ctypes.c_int]
    lib.bd_set_tail_mode.restype = ctypes.c_int
    lib.bd_set_graph_mode.argtypes = [V, ctypes.c_int]
    lib.bd_set_graph_mode.restype = ctypes.c_int
    lib.bd_set_stream.argtypes = [V, V]
    lib.bd_set_stream.restype = ctypes.c_int
    lib.bd_enable_kernel_timing.argtypes = [V, ctypes.c_int]
    lib.bd_enable_kernel_timing.restype = ctypes.c_int
    lib.bd_kernel_time.argtypes = [V, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.bd_kernel_time.restype = ctypes.c_int
    lib.bd_adjoint_begin.argtypes = [V, ctypes.c_int64, ctypes.c_int32]
    lib.bd_adjoint_begin.restype = ctypes.c_int
    lib.bd_adjoint_backward.argtypes = [V, V, V, V]
    lib.bd_adjoint_backward.restype = ctypes.c_int
    lib.bd_adjoint_backward_dev.argtypes = [V, V, V, V]
    lib.bd_adjoint_backward_dev.restype = ctypes.c_int
    lib.bd_get_state_dev.argtypes = [V, V, V]
    lib.bd_get_state_dev.restype = ctypes.c_int
    lib.bd_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, V]
    lib.bd_set_allocator.restype = ctypes.c_int
    lib.bd_destroy.argtypes = [V]
    lib.bd_destroy.restype = None
    lib.bd_batch_step.argtypes = [V, ctypes.c_int64]
    lib.bd_batch_step.restype = ctypes.c_int
    lib.bd_batch_get_state.argtypes = [V, V, V, P(ctypes.c_int64), P(Stats)]
    lib.bd_batch_get_state.restype = ctypes.c_int
    lib.bd_batch_destroy.argtypes = [V]
    lib.bd_batch_destroy.restype = None
    lib.bd_rollout.argtypes = [V, ctypes.c_int64, ctypes.c_int64]
    lib.bd_rollout.restype = ctypes.c_int
    lib.bd_backward.argtypes = [V, V, V, V]
    lib.bd_backward.restype = ctypes.c_int
    lib.bd_backward_dev.argtypes = [V, V, V, V]
    lib.bd_backward_dev.restype = ctypes.c_int
    lib.bd_pair_forces_dev.argtypes = [ctypes.c_int32, V, V, P(ForceParams), ctypes.c_int32, V, V]
    lib.bd_pair_forces_dev.restype = ctypes.c_int
    lib.bd_pair_forces_dev_noalloc.argtypes = [ctypes.c_int32, V, V, P(ForceParams), ctypes.c_int32, V, V]
    lib.bd_pair_forces_dev_noalloc.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def pair_forces_dev(xy, species, K, kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0, fp32=False, out=None,
                    noalloc=False):
    """Pair forces of torch CUDA tensors through bd_pair_forces_dev (or, noalloc=True, through
    bd_pair_forces_dev_noalloc, which only enqueues on torch's current stream): xy (n, 2) float64, species
    (n,) int32, K (S, S) host array.  Returns out, an (n, 2) float64 CUDA tensor (allocated here when None)."""
    import torch

    lib = load()
    if xy.dtype != torch.float64 or not xy.is_cuda or not xy.is_contiguous() or xy.dim() != 2 or xy.shape[1] != 2:
        raise ValueError("xy must be a contiguous (n, 2) float64 CUDA tensor")
    if species.dtype != torch.int32 or not species.is_cuda or not species.is_contiguous():
        raise ValueError("species must be a contiguous int32 CUDA tensor")
    n = xy.shape[0]
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float64, device=xy.device)
    Km = np.ascontiguousarray(K, dtype=np.float64)
    fp = ForceParams(BD_FORCE_POWER if kind == "power" else BD_FORCE_SCREENED, Km.shape[0], q, A, lam, cutoff,
                     0.0, _ptr(Km))
    stream = torch.cuda.current_stream(xy.device).cuda_stream
    fn = lib.bd_pair_forces_dev_noalloc if noalloc else lib.bd_pair_forces_dev
    rc = fn(n, xy.data_ptr(), species.data_ptr(), ctypes.byref(fp), BD_PREC_FP32 if fp32 else BD_PREC_FP64,
            out.data_ptr(), stream)
    if rc != 0:
        raise BDError(rc, f"{fn.__name__} failed: {lib.bd_strerror(rc).decode()}")
    return out


def _params(lib, *, L, kind, q, A, lam, cutoff, skin, K, D, dt, v0, Dr, seed, step0, overlap_factor, cap_frac,
            noise_clip, contact_tol, max_overlap_rounds, max_flip_rounds, fp32, force_chunk, force_per_lane,
            force_launch, overlap, max_dt_halvings, periodic):
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
    p.force_chunk = force_chunk
    p.force_per_lane, p.force_launch = force_per_lane, force_launch
    p.overlap_method = {"delaunay": BD_OVERLAP_DELAUNAY, "verlet": BD_OVERLAP_VERLET}[overlap]
    p.max_dt_halvings = max_dt_halvings
    p.periodic = 1 if periodic else 0
    return fp, p, Km


_DEFAULTS = dict(kind="power", q=2.0, A=1.0, lam=0.5, cutoff=0.0, skin=0.0, D=1.0, dt=1e-4, v0=0.0, Dr=0.0, seed=0,
                 step0=0, overlap_factor=1.0, cap_frac=0.5, noise_clip=3.0, contact_tol=1e-9,
                 max_overlap_rounds=10000, max_flip_rounds=200, fp32=False, force_chunk=0, force_per_lane=0,
                 force_launch=0, overlap="delaunay", max_dt_halvings=0, periodic=False)


class Sim:
    """One simulation handle (``bd_sim``) living on the current HIP device."""

    def __init__(self, xy, radii, species, theta, K, *, L, **kw):
        lib = load()
        self._lib = lib
        opts = dict(_DEFAULTS)
        opts.update(kw)
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self.n = xy.shape[0]
        rad = np.ascontiguousarray(radii, dtype=np.float64)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        fp, p, _keep = _params(lib, L=L, K=K, **opts)
        self._S = int(fp.S)
        h = ctypes.c_void_p()
        rc = lib.bd_init(ctypes.byref(h), self.n, _ptr(xy), _ptr(rad), _ptr(sp), None if th is None else _ptr(th),
                         ctypes.byref(fp), ctypes.byref(p))
        if rc != 0:
            raise BDError(rc, f"bd_init failed: {lib.bd_strerror(rc).decode()}")
        self._h = h

    @classmethod
    def batch(cls, xys, radii, species, thetas, Ls, seeds, K, **kw):
        """R independent systems in one handle (``bd_batch_init``); lists hold one entry per system."""
        self = cls.__new__(cls)
        lib = load()
        self._lib = lib
        opts = dict(_DEFAULTS)
        opts.update(kw)
        R = len(xys)
        n_per = np.array([len(np.asarray(a).reshape(-1, 2)) for a in xys], dtype=np.int32)
        xy = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1, 2) for a in xys]))
        rad = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64) for a in radii]))
        sp = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.int32) for a in species]))
        th = None
        if thetas is not None:
            th = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64) for a in thetas]))
        L_per = np.ascontiguousarray(Ls, dtype=np.float64)
        seed_per = np.ascontiguousarray([int(v) & (2**64 - 1) for v in seeds], dtype=np.uint64)
        self.n = int(n_per.sum())
        fp, p, _keep = _params(lib, L=float(L_per[0]), K=K, **opts)
        self._S = int(fp.S)
        h = ctypes.c_void_p()
        rc = lib.bd_batch_init(ctypes.byref(h), R, _ptr(n_per), _ptr(xy), _ptr(rad), _ptr(sp),
                               None if th is None else _ptr(th), _ptr(L_per), _ptr(seed_per), ctypes.byref(fp),
                               ctypes.byref(p))
        if rc != 0:
            raise BDError(rc, f"bd_batch_init failed: {lib.bd_strerror(rc).decode()}")
        self._h = h
        return self

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(L=w.L, kind=w.kind, q=w.q, A=w.A, lam=w.lam, cutoff=w.cutoff, skin=w.skin, D=w.D, dt=w.dt,
                  v0=w.v0, Dr=w.Dr, seed=w.seed, step0=w.step0, overlap_factor=w.overlap_factor,
                  cap_frac=w.cap_frac, noise_clip=w.noise_clip, contact_tol=w.contact_tol,
                  max_overlap_rounds=w.max_overlap_rounds, fp32=w.fp32_forces, overlap=w.overlap,
                  max_dt_halvings=w.max_dt_halvings, periodic=getattr(w, "periodic", False))
        kw.update(over)
        return cls(w.xy, w.radii, w.species, w.theta, w.K, **kw)

    @classmethod
    def from_workloads(cls, ws, **over):
        """Batch of workloads that share force and step parameters (box sides and seeds per system)."""
        w = ws[0]
        kw = dict(kind=w.kind, q=w.q, A=w.A, lam=w.lam, cutoff=w.cutoff, skin=w.skin, D=w.D, dt=w.dt, v0=w.v0,
                  Dr=w.Dr, step0=w.step0, overlap_factor=w.overlap_factor, cap_frac=w.cap_frac,
                  noise_clip=w.noise_clip, contact_tol=w.contact_tol, max_overlap_rounds=w.max_overlap_rounds,
                  fp32=w.fp32_forces)
        kw.update(over)
        return cls.batch([v.xy for v in ws], [v.radii for v in ws], [v.species for v in ws],
                         [v.theta for v in ws] if all(v.theta is not None for v in ws) else None,
                         [v.L for v in ws], [v.seed for v in ws], w.K, **kw)

    def layout(self):
        """(R, disk_off[R+1], frame_off[R+1]) of ``bd_batch_layout``."""
        R = ctypes.c_int32()
        self._check(self._lib.bd_batch_layout(self._h, ctypes.byref(R), None, None), "bd_batch_layout")
        d = np.zeros(R.value + 1, dtype=np.int32)
        f = np.zeros(R.value + 1, dtype=np.int32)
        self._check(self._lib.bd_batch_layout(self._h, ctypes.byref(R), _ptr(d), _ptr(f)), "bd_batch_layout")
        return R.value, d, f

    def force_config(self):
        c = ForceConfig()
        self._check(self._lib.bd_get_force_config(self._h, ctypes.byref(c)), "bd_get_force_config")
        return c.as_dict()

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

    def set_graph_mode(self, on: bool = True):
        self._check(self._lib.bd_set_graph_mode(self._h, 1 if on else 0), "bd_set_graph_mode")

    def set_tail_mode(self, mode: int):
        """0: one launch per phase; 1: overlap rounds after the first detection in one workgroup; -1: automatic."""
        self._check(self._lib.bd_set_tail_mode(self._h, int(mode)), "bd_set_tail_mode")

    def set_stream(self, stream_handle: Optional[int]):
        self._check(self._lib.bd_set_stream(self._h, stream_handle), "bd_set_stream")

    def enable_kernel_timing(self, on: bool = True):
        self._check(self._lib.bd_enable_kernel_timing(self._h, 1 if on else 0), "bd_enable_kernel_timing")

    def kernel_time(self):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self._lib.bd_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(cnt)), "bd_kernel_time")
        return float(ms.value), int(cnt.value)

    def adjoint_begin(self, nsteps: int, checkpoint_every: int):
        """Advance nsteps steps keeping checkpoints for ``adjoint_backward``."""
        self._check(self._lib.bd_adjoint_begin(self._h, int(nsteps), int(checkpoint_every)), "bd_adjoint_begin")

    def state_dev(self, xy_out: int, theta_out: int = 0):
        """Positions and angles into device buffers (raw device pointers, e.g. ``tensor.data_ptr()``)."""
        self._check(self._lib.bd_get_state_dev(self._h, xy_out or None, theta_out or None), "bd_get_state_dev")

    def adjoint_backward_dev(self, grad_xy: int, grad_xy0: int, grad_K: int):
        """``adjoint_backward`` on device buffers (raw device pointers)."""
        self._check(self._lib.bd_adjoint_backward_dev(self._h, grad_xy, grad_xy0 or None, grad_K or None),
                    "bd_adjoint_backward_dev")

    def adjoint_backward(self, grad_xy):
        """dL/dx at the first step and dL/dK from dL/dx at the last step of ``adjoint_begin``."""
        g = np.ascontiguousarray(grad_xy, dtype=np.float64).reshape(-1, 2)
        g0 = np.zeros((self.n, 2), dtype=np.float64)
        S = self._S
        gK = np.zeros((S, S), dtype=np.float64)
        self._check(self._lib.bd_adjoint_backward(self._h, _ptr(g), _ptr(g0), _ptr(gK)), "bd_adjoint_backward")
        return g0, gK

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
