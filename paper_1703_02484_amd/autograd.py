"""``torch.autograd.Function`` over the library's rollout and its adjoint sweep.

``rollout(K, x0, spec, nsteps, every)`` returns the positions after ``nsteps``
steps that start from positions ``x0`` with strength matrix ``K``; its
backward is ``bd_adjoint_backward`` (gradients with respect to ``K`` and
``x0`` with the overlap correction treated as a projection, checkpoints every
``every`` steps and recomputation in between).  Argument marshalling only:
the steps and the sweep run in ``libbd.so``.  Tensors are float64 on the host.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding


@dataclass
class RolloutSpec:
    """Everything of a system except K and the initial positions."""
    radii: np.ndarray
    species: np.ndarray
    theta: np.ndarray | None
    params: dict = field(default_factory=dict)   # keyword arguments of ``binding.Sim`` (L, D, dt, seed, ...)

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(L=w.L, kind=w.kind, q=w.q, A=w.A, lam=w.lam, cutoff=w.cutoff, skin=w.skin, D=w.D, dt=w.dt,
                  v0=w.v0, Dr=w.Dr, seed=w.seed, step0=w.step0, overlap_factor=w.overlap_factor,
                  cap_frac=w.cap_frac, noise_clip=w.noise_clip, contact_tol=w.contact_tol,
                  max_overlap_rounds=w.max_overlap_rounds, fp32=w.fp32_forces)
        kw.update(over)
        return cls(np.asarray(w.radii), np.asarray(w.species), None if w.theta is None else np.asarray(w.theta), kw)


class Rollout(torch.autograd.Function):
    """Host tensors go through host copies; CUDA tensors (float64, on the handle's GPU) are read and
    written in place through the device-pointer entry points."""

    @staticmethod
    def forward(ctx, K, x0, spec, nsteps, every):
        sim = binding.Sim(x0.detach().cpu().numpy(), spec.radii, spec.species, spec.theta,
                          K.detach().cpu().numpy(), **spec.params)
        sim.adjoint_begin(int(nsteps), int(every))
        ctx.sim = sim
        if x0.is_cuda:
            xT = torch.empty(x0.shape, dtype=torch.float64, device=x0.device)
            torch.cuda.current_stream(x0.device).synchronize()   # xT's memory is free on torch's stream
            sim.state_dev(xT.data_ptr())
            return xT
        return torch.from_numpy(sim.state()[0])

    @staticmethod
    def backward(ctx, grad):
        if grad.is_cuda:
            g = grad.detach().to(torch.float64).contiguous()
            g0 = torch.empty_like(g)
            S = ctx.sim._S
            gK = torch.empty((S, S), dtype=torch.float64, device=g.device)
            torch.cuda.current_stream(g.device).synchronize()   # grad is complete before the library reads it
            ctx.sim.adjoint_backward_dev(g.data_ptr(), g0.data_ptr(), gK.data_ptr())
            return gK, g0, None, None, None
        g0, gK = ctx.sim.adjoint_backward(grad.detach().cpu().contiguous().numpy())
        return torch.from_numpy(gK), torch.from_numpy(g0), None, None, None


def rollout(K: torch.Tensor, x0: torch.Tensor, spec: RolloutSpec, nsteps: int, every: int = 10) -> torch.Tensor:
    """Positions (n, 2) after ``nsteps`` steps; differentiable in ``K`` (S, S) and ``x0`` (n, 2)."""
    return Rollout.apply(K, x0, spec, nsteps, every)


def msd_loss(xT: torch.Tensor, x0: torch.Tensor, species: np.ndarray, s: int = 0) -> torch.Tensor:
    """Mean squared displacement of the particles of species s."""
    mask = torch.from_numpy(np.asarray(species) == s).to(xT.device)
    d = xT[mask] - x0[mask]
    return (d * d).sum() / mask.sum()
