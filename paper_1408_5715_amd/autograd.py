"""Differentiable rollouts of the FV step: a torch.autograd.Function whose
forward runs the library's step and whose backward runs the library's
adjoint step (fv_step_adjoint / fv_step_adjoint_grad), with checkpointing.

Memory: the forward keeps one state every `checkpoint` steps (plus the
states it returns); the backward recomputes the states inside each segment
from its checkpoint (at most `checkpoint` of them at a time) and walks the
adjoint back through them.  With correction parameters, the forward sets
them on the solver and the backward also returns their gradient.  Torch only
provides device memory; every step and adjoint step runs in the HIP library.
"""

from __future__ import annotations

import numpy as np
import torch

from .fvgpu import (FV_CORRECTION_PARAMS, fv_step, fv_step_adjoint_grad, fv_upload_state_device)


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, params, solver, n_steps: int, dt: float, checkpoint: int = 4,
                every: int = 0):
        if U0.dtype != torch.float64 or U0.shape != (solver.n, 4) or not U0.is_cuda:
            raise ValueError("U0 must be a float64 CUDA tensor of shape [n_cells, 4]")
        if n_steps < 1:
            raise ValueError("n_steps must be >= 1")
        checkpoint = max(1, int(checkpoint))
        every = int(every) if every else n_steps
        if n_steps % every:
            raise ValueError("every must divide n_steps")
        if isinstance(dt, (list, tuple, np.ndarray, torch.Tensor)):
            raise ValueError("a rollout takes one dt for every mesh (the adjoint step has one)")
        dt = float(dt)
        p = None
        if params is not None:
            p = params.detach().to("cpu", torch.float32).numpy().copy()
            if p.shape != (FV_CORRECTION_PARAMS,):
                raise ValueError(f"params must have {FV_CORRECTION_PARAMS} values")
        # the rollout runs the plain step without params, whatever the
        # solver held before; the backward sets the same correction again
        solver.set_correction(p)
        fv_upload_state_device(solver.ctx, U0.contiguous())
        saved, outs = [], []
        for s in range(n_steps):
            if s % checkpoint == 0:
                saved.append(solver.download_device())  # state at step s
            fv_step(solver.ctx, 1, dt)
            if (s + 1) % every == 0:
                outs.append(solver.download_device())
        ctx.solver, ctx.n_steps, ctx.dt = solver, n_steps, dt
        ctx.checkpoint, ctx.every, ctx.saved = checkpoint, every, saved
        ctx.with_params = params is not None
        ctx.params_host = p
        ctx.params_device = params.device if params is not None else None
        out = torch.stack(outs) if every != n_steps else outs[0]
        return out

    @staticmethod
    def backward(ctx, grad_out):
        s, dt, cp, every = ctx.solver, ctx.dt, ctx.checkpoint, ctx.every
        n = ctx.n_steps
        grads = grad_out if every != n else grad_out[None]
        lam = torch.zeros((s.n, 4), dtype=torch.float64, device=grad_out.device)
        gtheta = (torch.zeros(FV_CORRECTION_PARAMS, dtype=torch.float64, device=grad_out.device)
                  if ctx.with_params else None)
        # the solver may have been given another correction since the forward
        s.set_correction(ctx.params_host)
        starts = list(range(0, n, cp))
        for seg, start in reversed(list(enumerate(starts))):
            k = min(cp, n - start)
            states = [ctx.saved[seg]]
            fv_upload_state_device(s.ctx, ctx.saved[seg])
            for _ in range(k - 1):
                fv_step(s.ctx, 1, dt)
                states.append(s.download_device())
            for i in reversed(range(k)):
                step = start + i  # this step maps U^step to U^(step+1)
                if (step + 1) % every == 0:
                    lam += grads[(step + 1) // every - 1]
                fv_step_adjoint_grad(s.ctx, states[i], lam, dt, gtheta)
        ctx.saved = None
        ctx.params_host = None
        gp = None
        if ctx.with_params:
            gp = gtheta.to(ctx.params_device, torch.float32)
        return lam, gp, None, None, None, None, None


def rollout(U0, solver, n_steps: int, dt: float, checkpoint: int = 4, params=None,
            every: int = 0):
    """States after a rollout of n_steps steps from U0 (float64 CUDA [n, 4],
    mesh numbering), differentiable with respect to U0 and, if given, the
    correction parameters (float32 [FV_CORRECTION_PARAMS], set on the solver
    for the rollout; without them the plain step runs).  dt is one time step
    for every mesh of a batch.  every = 0: the final state; else the states after
    every `every` steps, stacked [n_steps / every, n, 4]."""
    return Rollout.apply(U0, params, solver, n_steps, dt, checkpoint, every)
