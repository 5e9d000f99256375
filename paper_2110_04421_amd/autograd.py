"""``torch.autograd.Function`` over the relaxed (Gumbel-softmax) simulator.

The forward pass runs the relaxed day loop of the library on the GPU for parameters
theta = (R, S_0..S_8) per replicate and returns the daily relaxed incidence [R, days].
The backward pass is the library's hand-written adjoint (``abm_grad``): a reverse sweep
over the checkpointed days, so that d loss / d theta costs about three forward passes
and no graph is recorded.  Section 1 and section 6 of the paper motivate differentiable
calibration; the relaxation and the adjoint are this implementation's.

    theta = torch.tensor(..., requires_grad=True)        # [replicates, 10]
    c = relaxed_incidence(theta, params, pop, days)      # [replicates, days]
    loss = ((c - target) ** 2).sum(); loss.backward()    # theta.grad via abm_grad
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib as L


class RelaxedIncidence(torch.autograd.Function):
    """theta [R, 10] -> relaxed daily incidence [R, days] (float32)."""

    @staticmethod
    def forward(ctx, theta, params, pop, days):
        from .sim import Simulator
        th = theta.detach().to("cpu", torch.float64).numpy()
        if th.shape != (pop.n_replicates, L.N_THETA):
            raise ValueError(f"theta must be [{pop.n_replicates}, {L.N_THETA}], got {tuple(th.shape)}")
        q = dataclasses.replace(pop, R=th[:, 0].astype(np.float32),
                                susceptibility=np.ascontiguousarray(th[:, 1:], np.float32))
        sim = Simulator(dict(params, mode=L.SOFT, n_steps=int(days)), q)
        c = sim.run(int(days))
        ctx.sim = sim                 # holds the checkpoints the adjoint sweeps back over
        ctx.meta = (theta.dtype, theta.device)
        return torch.from_numpy(c).to(theta.device)

    @staticmethod
    def backward(ctx, grad_c):
        sim = ctx.sim
        dtype, device = ctx.meta
        g = sim.grad(grad_c.detach().to("cpu", torch.float32).numpy())
        sim.close()
        ctx.sim = None
        return torch.from_numpy(g).to(device=device, dtype=dtype), None, None, None


def relaxed_incidence(theta, params: dict, pop, days: int):
    """Relaxed daily incidence [R, days] of ``pop`` at parameters ``theta`` [R, 10];
    differentiable in theta through the library's adjoint."""
    return RelaxedIncidence.apply(theta, params, pop, days)


ABMFunction = RelaxedIncidence
