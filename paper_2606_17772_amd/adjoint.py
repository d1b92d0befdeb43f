"""Differentiable FD-CGKS time stepping on top of fdcgks_step_vjp.

The reverse pass never differentiates through kernels traced by PyTorch: the
vector-Jacobian product of a step is the library's hand-written adjoint
(include/fdcgks.h, fdcgks_step_vjp), evaluated at a fixed time step.  These
autograd functions only save states (checkpoints) and call forward steps and
step adjoints in the right order.

    S = get_state_vector(problem, device="cuda")   # float64 state of both grids
    S.requires_grad_(True)
    out = rollout(problem, S, dt=1e-3, nsteps=50, checkpoint_every=8)
    J = 0.5 * ((density(problem, out) - rho_target) ** 2).sum() * h * h
    J.backward()                                    # S.grad = dJ/dS

States: on periodic problems the stacked (2, 12, ny, nx) tensor
(get_state_all); with a bounded axis the grids differ in size and a state
is the flat vector of grid 0's 12 planes followed by grid 1's (the C ABI's
layout).  get_state_vector / set_state_vector give either form.

Checkpointing: `rollout` keeps only every `checkpoint_every`-th state; the
backward pass recomputes the states inside a segment from its checkpoint
(forward steps), then walks the segment backwards with one step adjoint per
step.  Memory: (nsteps / every + every) states instead of nsteps.
"""
from __future__ import annotations

import torch

__all__ = ["step", "rollout", "get_state_vector", "set_state_vector", "density"]


def _grid_sizes(problem):
    """Elements of each grid's W, Wx, Wy planes."""
    return [3 * int(torch.Size(problem.grid_shape(g)).numel()) for g in range(problem.ngrid)]


def get_state_vector(problem, device):
    """The current state as a torch tensor on `device`: stacked (periodic)
    or flat (bounded axes)."""
    if not any(problem.bounded):
        return problem.get_state_all(device=device)
    return torch.cat([a.reshape(-1) for g in range(problem.ngrid) for a in problem.get_state(g, device)])


def set_state_vector(problem, S):
    """Set the state from a tensor of get_state_vector's form."""
    S = S.detach().contiguous()
    if not any(problem.bounded):
        problem.set_state_all(S)
        return
    off = 0
    for g, n3 in enumerate(_grid_sizes(problem)):
        n = n3 // 3
        problem.set_state(g, S[off:off + n], S[off + n:off + 2 * n], S[off + 2 * n:off + n3])
        off += n3


def density(problem, S):
    """The primary grid's density plane (ny, nx) of a state of either form."""
    if not any(problem.bounded):
        return S[0, 0]
    p = problem.params
    return S[:p.nx * p.ny].reshape(p.ny, p.nx)


def _vjp(problem, dt, lam):
    lam = lam.contiguous()
    if not any(problem.bounded):
        return problem.step_vjp(dt, lam)
    sizes = _grid_sizes(problem)
    parts = [q.reshape((3 * problem.ncomp,) + tuple(problem.grid_dims(g)))
             for g, q in enumerate(torch.split(lam, sizes))]
    return torch.cat([a.reshape(-1) for a in problem.step_vjp(dt, parts)])


def _run(problem, S, dt, nsteps):
    set_state_vector(problem, S)
    if nsteps:
        problem.step(nsteps=nsteps, dt=dt)
    return get_state_vector(problem, S.device)


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
        set_state_vector(ctx.problem, S)
        return _vjp(ctx.problem, ctx.dt, lam), None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, problem, dt, nsteps, every):
        ckpts = [S.detach().clone()]
        set_state_vector(problem, ckpts[0])
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            problem.step(nsteps=k, dt=dt)
            done += k
            if done < nsteps:
                ckpts.append(get_state_vector(problem, S.device))
        out = get_state_vector(problem, S.device)
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
                set_state_vector(pb, s)
                lam = _vjp(pb, dt, lam)
        return lam, None, None, None, None


def step(problem, S, dt):
    """One step of size dt from the state S (get_state_vector's form); the
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
