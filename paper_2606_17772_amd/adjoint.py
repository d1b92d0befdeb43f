"""Differentiable FD-CGKS time stepping on top of fdcgks_step_vjp.

The reverse pass never differentiates through kernels traced by PyTorch: the
vector-Jacobian product of a step is the library's hand-written adjoint
(include/fdcgks.h, fdcgks_step_vjp), evaluated at a fixed time step.  These
autograd functions only save states (checkpoints) and call forward steps and
step adjoints in the right order.

    S = torch.as_tensor(stacked_state, device="cuda")   # (2, 12, ny, nx) float64
    S.requires_grad_(True)
    out = rollout(problem, S, dt=1e-3, nsteps=50, checkpoint_every=8)
    J = 0.5 * ((out[0, 0] - rho_target) ** 2).sum() * h * h
    J.backward()                                          # S.grad = dJ/dS

Checkpointing: `rollout` keeps only every `checkpoint_every`-th state; the
backward pass recomputes the states inside a segment from its checkpoint
(forward steps), then walks the segment backwards with one step adjoint per
step.  Memory: (nsteps / every + every) states instead of nsteps.
"""
from __future__ import annotations

import torch

__all__ = ["step", "rollout"]


def _run(problem, S, dt, nsteps):
    problem.set_state_all(S.detach().contiguous())
    if nsteps:
        problem.step(nsteps=nsteps, dt=dt)
    return problem.get_state_all(device=S.device)


class _Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, problem, dt):
        out = _run(problem, S, dt, 1)
        ctx.save_for_backward(S.detach())
        ctx.problem, ctx.dt = problem, dt
        return out

    @staticmethod
    def backward(ctx, lam):
        (S,) = ctx.saved_tensors
        ctx.problem.set_state_all(S.contiguous())
        return ctx.problem.step_vjp(ctx.dt, lam.contiguous()), None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, problem, dt, nsteps, every):
        ckpts = [S.detach().clone()]
        problem.set_state_all(ckpts[0].contiguous())
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            problem.step(nsteps=k, dt=dt)
            done += k
            if done < nsteps:
                ckpts.append(problem.get_state_all(device=S.device))
        out = problem.get_state_all(device=S.device)
        ctx.save_for_backward(*ckpts)
        ctx.problem, ctx.dt, ctx.nsteps, ctx.every = problem, dt, nsteps, every
        return out

    @staticmethod
    def backward(ctx, lam):
        pb, dt, every = ctx.problem, ctx.dt, ctx.every
        ckpts = ctx.saved_tensors
        lam = lam.contiguous()
        for seg in reversed(range(len(ckpts))):
            k = min(every, ctx.nsteps - seg * every)
            # states at the start of every step of the segment
            states = [ckpts[seg]]
            for _ in range(k - 1):
                states.append(_run(pb, states[-1], dt, 1))
            for s in reversed(states):
                pb.set_state_all(s.contiguous())
                lam = pb.step_vjp(dt, lam)
        return lam, None, None, None, None


def step(problem, S, dt):
    """One step of size dt from the stacked state S (2, 12, ny, nx); the
    result is differentiable with respect to S."""
    return _Step.apply(S, problem, float(dt))


def rollout(problem, S, dt, nsteps, checkpoint_every=None):
    """nsteps steps of size dt from S with segment checkpointing (default
    segment length: about sqrt(nsteps))."""
    nsteps = int(nsteps)
    if nsteps < 1:
        raise ValueError("nsteps must be >= 1")
    every = int(checkpoint_every) if checkpoint_every else max(1, int(round(nsteps ** 0.5)))
    return _Rollout.apply(S, problem, float(dt), nsteps, every)
