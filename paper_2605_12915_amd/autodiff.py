"""Differentiation form: torch.autograd.Function wrappers around af_step_out and
af_step_adjoint, and a checkpointed multi-step rollout.

The forward and the reverse steps run in libaf.so's kernels; this module only
orchestrates which state each call receives (checkpoint every `checkpoint_every`
steps, recompute the states of a segment, then step backwards through it).
"""
from __future__ import annotations

import torch

from .stepper import Stepper


class AFStep(torch.autograd.Function):
    """One step, state_n -> state_{n+1}; backward = af_step_adjoint (dt fixed)."""

    @staticmethod
    def forward(ctx, state: torch.Tensor, stepper: Stepper, dt: float):
        out = stepper.step_out(state.detach(), dt)
        ctx.save_for_backward(state.detach())
        ctx.stepper, ctx.dt = stepper, dt
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (state,) = ctx.saved_tensors
        g = ctx.stepper.adjoint(state, grad_out.contiguous(), ctx.dt)
        return g, None, None


class AFRollout(torch.autograd.Function):
    """nsteps steps with checkpoints every `every` steps; memory O(nsteps/every + every)
    states; the backward pass recomputes each segment once from its checkpoint."""

    @staticmethod
    def forward(ctx, state0: torch.Tensor, stepper: Stepper, dt: float, nsteps: int, every: int):
        x = state0.detach().clone()
        ckpts = [x.clone()]
        for s in range(nsteps):
            x = stepper.step_out(x, dt)
            if (s + 1) % every == 0 and s + 1 < nsteps:
                ckpts.append(x.clone())
        ctx.ckpts, ctx.stepper, ctx.dt, ctx.nsteps, ctx.every = ckpts, stepper, dt, nsteps, every
        return x

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        st, dt, n, k = ctx.stepper, ctx.dt, ctx.nsteps, ctx.every
        g = g.contiguous()
        nseg = len(ctx.ckpts)
        for seg in reversed(range(nseg)):
            start = seg * k
            stop = min(n, start + k)
            states = [ctx.ckpts[seg]]
            for _ in range(start, stop - 1):
                states.append(st.step_out(states[-1], dt))
            for s in reversed(range(stop - start)):
                g = st.adjoint(states[s], g, dt)
        return g, None, None, None, None


def step(state: torch.Tensor, stepper: Stepper, dt: float) -> torch.Tensor:
    return AFStep.apply(state, stepper, dt)


def rollout(state0: torch.Tensor, stepper: Stepper, dt: float, nsteps: int, checkpoint_every: int = 20):
    return AFRollout.apply(state0, stepper, dt, nsteps, checkpoint_every)
