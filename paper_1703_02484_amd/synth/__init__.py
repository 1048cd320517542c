"""Seeded synthetic workloads for the Brownian hard-disk step.

This module only generates inputs (initial positions, radii, species, initial
director angles and parameter sets).  It contains none of the method's
arithmetic and is shared by the GPU library's tests and benchmark and by the
CPU oracle's tests.

The paper generates its own inputs (a lattice subsample, Sec. 4.1) and uses no
public dataset; its configuration table is not available.  The workloads here
are the synthetic stand-ins named C1..C5:

* positions: random sequential insertion of radius-1 disks, uniform centres in
  [r, L-r]^2, rejection on centre distance < 2r (``rsa.c``);
* box side from the paper's L(N) relation of Sec. 6 with the area fraction
  phi = N pi r^2 / L^2;
* species ``i mod S``; initial director angles uniform in [0, 2 pi).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_rsa.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the RSA generator into ``_rsa.so`` (plain C, gcc)."""
    src = os.path.join(_HERE, "rsa.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.rsa_disks.restype = ctypes.c_int
        lib.rsa_disks.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_longlong, ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]
        lib.rsa_disks_periodic.restype = ctypes.c_int
        lib.rsa_disks_periodic.argtypes = lib.rsa_disks.argtypes
        _lib = lib
    return _lib


def box_side(n: int, phi: float, r: float = 1.0) -> float:
    """Square box side for n disks of radius r at area fraction phi."""
    return math.sqrt(n * math.pi * r * r / phi)


def rsa(n: int, L: float, r: float = 1.0, seed: int = 0, max_attempts: Optional[int] = None,
        periodic: bool = False) -> np.ndarray:
    """Random sequential insertion of n disks of radius r into [0, L]^2 (hard walls: centres in [r, L-r]^2;
    periodic: centres in [0, L)^2, nearest-image separations); returns (n, 2) float64."""
    lib = _load()
    out = np.zeros((max(n, 0), 2), dtype=np.float64)
    if max_attempts is None:
        max_attempts = max(1000, 20000 * max(n, 1))
    att = ctypes.c_longlong(0)
    fn = lib.rsa_disks_periodic if periodic else lib.rsa_disks
    rc = fn(int(n), float(L), float(r), ctypes.c_uint64(seed & (2**64 - 1)), int(max_attempts),
            out.ctypes.data, ctypes.byref(att))
    if rc != 0:
        raise RuntimeError(f"rsa_disks failed rc={rc} (n={n}, L={L}, attempts={att.value})")
    return out


@dataclass
class Workload:
    """One synthetic configuration: arrays plus physical and numerical parameters."""
    name: str
    xy: np.ndarray            # (n, 2) float64
    radii: np.ndarray         # (n,) float64
    species: np.ndarray       # (n,) int32
    theta: np.ndarray         # (n,) float64
    S: int
    K: np.ndarray             # (S, S) float64, K[a, b] acts on species a from species b
    kind: str = "power"       # "power" (g = d^-q) or "screened" (g = A exp(-d/lam) / d)
    q: float = 2.0
    A: float = 1.0
    lam: float = 0.5
    cutoff: float = 0.0       # <= 0: all pairs
    skin: float = 0.0
    L: float = 0.0
    D: float = 1.0
    dt: float = 1e-4
    v0: float = 0.0
    Dr: float = 0.0
    seed: int = 0
    step0: int = 0
    overlap_factor: float = 1.0
    cap_frac: float = 0.5
    noise_clip: float = 3.0
    contact_tol: float = 1e-9   # overlap when d < (r_i + r_j)(1 - contact_tol)
    max_overlap_rounds: int = 10000
    steps: int = 100
    fp32_forces: bool = False
    overlap: str = "delaunay"      # overlap test over Delaunay edges, or "verlet": over the neighbour lists
    max_dt_halvings: int = 0       # halvings of a step whose move reversed a Delaunay edge (0: count only)
    periodic: bool = False         # periodic box [0, L)^2 instead of hard walls
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])


def _thetas(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed + 0x7E7A))
    return rng.uniform(0.0, 2.0 * math.pi, size=n)


def make(name: str, n: Optional[int] = None, seed: int = 0, steps: Optional[int] = None,
         periodic: bool = False) -> Workload:
    """Build workload ``name`` in {C1, C2, C3, C5} (optionally at a reduced n).

    C1  plain method, FP64: phi=0.30, S=1, K=1e-2, inverse-square law, all pairs.
    C2  FP32 forces: phi=0.40, S=2 (i mod 2), non-reciprocal K, self-propulsion v0=1, Dr=1.
    C3  short range: phi=0.50, S=1, K=1, screened law A=1, lam=0.5, cutoff 2.5, skin 0.5.
    C5  differentiation: phi=0.35, S=2, K=1e-2 everywhere, contact factor 1/2, 50 steps.

    periodic: the same workload in a periodic box of the same side (the paper's own domain, Sec. 2.1):
    positions placed with nearest-image separations in [0, L)^2, no walls.
    """
    if periodic:
        w = make(name, n, seed, steps)
        w.xy = rsa(w.n, w.L, 1.0, seed, periodic=True)
        w.periodic = True
        w.name = w.name + "p"
        return w
    r = 1.0
    if name == "C1":
        n = 1024 if n is None else n
        phi = 0.30
        L = box_side(n, phi, r)
        xy = rsa(n, L, r, seed)
        return Workload("C1", xy, np.full(n, r), np.zeros(n, np.int32), np.zeros(n), 1,
                        np.array([[1e-2]]), L=L, D=1.0, dt=1e-4, seed=seed,
                        steps=100 if steps is None else steps, fp32_forces=False)
    if name == "C2":
        n = 65536 if n is None else n
        phi = 0.40
        L = box_side(n, phi, r)
        xy = rsa(n, L, r, seed)
        sp = (np.arange(n) % 2).astype(np.int32)
        K = np.array([[1e-2, -5e-3], [2e-3, 1e-2]])
        return Workload("C2", xy, np.full(n, r), sp, _thetas(n, seed), 2, K, L=L, D=1.0, dt=1e-4,
                        v0=1.0, Dr=1.0, seed=seed, steps=1000 if steps is None else steps,
                        fp32_forces=True)
    if name == "C3":
        n = 1048576 if n is None else n
        phi = 0.50
        L = box_side(n, phi, r)
        xy = rsa(n, L, r, seed)
        return Workload("C3", xy, np.full(n, r), np.zeros(n, np.int32), np.zeros(n), 1,
                        np.array([[1.0]]), kind="screened", A=1.0, lam=0.5, cutoff=2.5, skin=0.5,
                        L=L, D=1.0, dt=1e-4, seed=seed, steps=10000 if steps is None else steps,
                        fp32_forces=True)
    if name == "C5":
        n = 16384 if n is None else n
        phi = 0.35
        L = box_side(n, phi, r)
        xy = rsa(n, L, r, seed)
        sp = (np.arange(n) % 2).astype(np.int32)
        return Workload("C5", xy, np.full(n, r), sp, np.zeros(n), 2, np.full((2, 2), 1e-2), L=L,
                        D=1.0, dt=1e-4, seed=seed, overlap_factor=0.5,
                        steps=50 if steps is None else steps, fp32_forces=False)
    raise ValueError(f"unknown workload {name!r}")


def batch_sizes(R: int = 256, seed: int = 0, lo: int = 2048, hi: int = 32768) -> List[int]:
    """Replica sizes for the batched workload C4: floor(exp(U[ln lo, ln hi]))."""
    rng = np.random.Generator(np.random.PCG64(seed + 0xB47C4))
    u = rng.uniform(math.log(lo), math.log(hi), size=R)
    return [int(math.floor(math.exp(v))) for v in u]


def batch_phis(R: int = 256, seed: int = 0) -> List[float]:
    rng = np.random.Generator(np.random.PCG64(seed + 0xF1C4))
    return [float(v) for v in rng.uniform(0.2, 0.5, size=R)]


def make_batch(R: int = 256, seed: int = 0, lo: int = 2048, hi: int = 32768,
               steps: Optional[int] = None) -> List[Workload]:
    """Batched workload C4: R independent systems of the C1 kind (FP64, S=1, K=1e-2, all pairs).

    System r has N_r = floor(exp(U[ln lo, ln hi])) disks of radius 1 at area fraction phi_r ~ U[0.2, 0.5],
    placed by random sequential insertion, and noise key seed_r = r.
    """
    sizes = batch_sizes(R, seed, lo, hi)
    phis = batch_phis(R, seed)
    out = []
    for r in range(R):
        n, phi = sizes[r], phis[r]
        L = box_side(n, phi, 1.0)
        xy = rsa(n, L, 1.0, seed * 1000003 + r)
        out.append(Workload("C4", xy, np.ones(n), np.zeros(n, np.int32), np.zeros(n), 1, np.array([[1e-2]]),
                            L=L, D=1.0, dt=1e-4, seed=r, steps=500 if steps is None else steps,
                            fp32_forces=False, extra={"phi": phi, "replica": r}))
    return out
