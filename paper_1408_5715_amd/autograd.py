"""Differentiable rollouts of the FV step: a torch.autograd.Function whose
forward runs the library's step and whose backward runs the library's
adjoint step (fv_step_adjoint), with checkpointing.

Memory: the forward keeps one state every `checkpoint` steps; the backward
recomputes the states inside each segment from its checkpoint (at most
`checkpoint` of them at a time) and walks the adjoint back through them.
Torch only provides device memory; every step and adjoint step runs in the
HIP library.
"""

from __future__ import annotations

import torch

from .fvgpu import (fv_download_state_device, fv_step, fv_step_adjoint, fv_upload_state_device)


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, n_steps: int, dt: float, checkpoint: int = 4):
        if U0.dtype != torch.float64 or U0.shape != (solver.n, 4) or not U0.is_cuda:
            raise ValueError("U0 must be a float64 CUDA tensor of shape [n_cells, 4]")
        checkpoint = max(1, int(checkpoint))
        U0 = U0.contiguous()
        saved = []
        fv_upload_state_device(solver.ctx, U0)
        done = 0
        while done < n_steps:
            k = min(checkpoint, n_steps - done)
            saved.append(solver.download_device())  # state at step `done`
            fv_step(solver.ctx, k, dt)
            done += k
        out = solver.download_device()
        ctx.solver, ctx.n_steps, ctx.dt, ctx.checkpoint = solver, n_steps, dt, checkpoint
        ctx.saved = saved
        return out

    @staticmethod
    def backward(ctx, grad_out):
        s, dt, cp = ctx.solver, ctx.dt, ctx.checkpoint
        lam = grad_out.contiguous().clone()
        starts = list(range(0, ctx.n_steps, cp))
        for seg, start in reversed(list(enumerate(starts))):
            k = min(cp, ctx.n_steps - start)
            states = [ctx.saved[seg]]
            fv_upload_state_device(s.ctx, ctx.saved[seg])
            for _ in range(k - 1):
                fv_step(s.ctx, 1, dt)
                states.append(s.download_device())
            for U in reversed(states):
                fv_step_adjoint(s.ctx, U, lam, dt)
        ctx.saved = None
        return lam, None, None, None, None


def rollout(U0, solver, n_steps: int, dt: float, checkpoint: int = 4):
    """U after n_steps steps from U0 (float64 CUDA [n, 4], mesh numbering),
    differentiable with respect to U0."""
    return Rollout.apply(U0, solver, n_steps, dt, checkpoint)
