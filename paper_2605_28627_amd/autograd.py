"""Discrete adjoint of LSERK4(5) trajectories behind torch.autograd.

`trajectory(solver, U0, dt, nsteps)` returns U(T) and is differentiable with
respect to U0; the backward pass runs the library's hand-written adjoint over
the steps in reverse, recomputing the step states segment by segment from
checkpoints kept during the forward pass; the recomputation keeps each
step's stage states (dg_rk_step_stages) so that the reverse step
(dg_adjoint_rk_step_stages) need not recompute them.  `kinetic_energy(solver, U)` is the
paper's integral kinetic energy E_k and its gradient, both evaluated by the
library.  PyTorch is used for memory and the autograd graph only.
"""
from __future__ import annotations

import math

import torch

from . import dgx


# state-sized registers the trajectory holds besides the checkpoints and the
# recomputed states: the forward state and RK register, the input gradient,
# and in the backward pass lambda_U, lambda_dU, the RK register and the
# recomputation state
_EXTRA_STATES = 7


def checkpoint_plan(solver, nsteps: int, memory_fraction: float = 0.9, store_stages: bool = True) -> tuple[int, int]:
    """(k, j): checkpoints every k steps, and in each segment the stage states
    of j of its k-1 recomputed steps kept.  The backward pass then holds
    nsteps/k checkpoints, the k step states of a segment and j (S-1) stage
    states, and recomputes ((k-1) S + (k-j) (S-1)) / k residuals per step (the
    reverse step recomputes the stages it is not given).  The cheapest plan
    whose states (and the other state-sized registers) fit in a fraction of
    the free HBM is taken (torch's cached blocks count as free)."""
    state_bytes = solver.state_len * 8
    free, _ = torch.cuda.mem_get_info(solver.device)
    free += torch.cuda.memory_reserved(solver.device) - torch.cuda.memory_allocated(solver.device)
    budget = int(free * memory_fraction) // state_bytes - _EXTRA_STATES
    S = solver.rk_stages
    best = None
    for k in range(1, max(nsteps, 1) + 1):
        for j in range(0, (k - 1 if store_stages else 0) + 1):
            mem = math.ceil(nsteps / k) + k + j * (S - 1)
            if mem > budget:
                break
            key = (((k - 1) * S + (k - j) * (S - 1)) / k, mem)
            if best is None or key < best[0]:
                best = (key, (k, j))
    if best is None:
        k = max(1, int(math.ceil(math.sqrt(nsteps))))
        raise MemoryError(f"{nsteps} steps need at least {math.ceil(nsteps / k) + k + _EXTRA_STATES} states of "
                          f"{state_bytes / 2**30:.2f} GiB; about {int(free * memory_fraction) // state_bytes} fit")
    return best[1]


def checkpoint_interval(solver, nsteps: int, memory_fraction: float = 0.9, store_stages: bool = True) -> int:
    """Steps between checkpoints of checkpoint_plan."""
    return checkpoint_plan(solver, nsteps, memory_fraction, store_stages)[0]


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, nsteps, every, keep):
        U = U0.detach().clone()
        dU = torch.empty_like(U)
        ckpts = {}
        for n in range(nsteps):
            if n % every == 0:
                ckpts[n] = U.clone()
            solver.rk_step(U, dU, dt, 1)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.every, ctx.ckpts = solver, dt, nsteps, every, ckpts
        ctx.keep = keep
        return U

    @staticmethod
    def backward(ctx, grad_out):
        solver, dt, nsteps, every = ctx.solver, ctx.dt, ctx.nsteps, ctx.every
        lamU = grad_out.detach().contiguous().clone()
        lamdU = torch.empty_like(lamU)
        dU = torch.empty_like(lamU)
        starts = sorted(ctx.ckpts.keys())
        for s0 in reversed(starts):
            s1 = min(s0 + every, nsteps)
            # recompute the segment's step states (and, kept, their stage states)
            states, stages = [ctx.ckpts[s0]], []
            U = ctx.ckpts[s0].clone()
            for n in range(s0, s1 - 1):
                if n - s0 < ctx.keep:
                    Y = solver.stage_buffer()
                    solver.rk_step_stages(U, dU, dt, Y)
                    stages.append(Y)
                else:
                    solver.rk_step(U, dU, dt, 1)
                states.append(U.clone())
            for n in reversed(range(s0, s1)):
                if n - s0 < len(stages):
                    solver.adjoint_rk_step_stages(states[n - s0], stages[n - s0], lamU, lamdU, dt)
                else:   # (the segment's last step: its stages are recomputed)
                    solver.adjoint_rk_step(states[n - s0], lamU, lamdU, dt)
            del states, stages
        ctx.ckpts = None
        return lamU, None, None, None, None, None


def trajectory(solver, U0: torch.Tensor, dt: float, nsteps: int, checkpoint_every: int | None = None,
               keep_stages: int | None = None):
    """U(T) after nsteps LSERK steps of size dt; differentiable in U0.  The
    backward pass recomputes each segment of checkpoint_every steps from its
    checkpoint and keeps the stage states of its first keep_stages steps
    (both from checkpoint_plan unless given; no stage states in contexts with
    FV sub-cells)."""
    if not getattr(solver, "adjoint", False):
        raise ValueError("the solver was created without the adjoint workspace (DGSolver(..., adjoint=True))")
    store = not solver.cfg.get("fv", 0)
    if checkpoint_every is None:
        every, keep = checkpoint_plan(solver, nsteps, store_stages=store)
    else:
        every, keep = checkpoint_every, (checkpoint_every - 1 if store else 0)
    if keep_stages is not None:
        keep = min(keep_stages, every - 1) if store else 0
    return _Trajectory.apply(U0, solver, float(dt), int(nsteps), int(every), int(keep))


class _KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, solver, rho0U0sq):
        ctx.save_for_backward(U)
        ctx.solver, ctx.rho0U0sq = solver, rho0U0sq
        out = torch.empty(1, dtype=torch.float64, device=U.device)
        dgx.dg_kinetic_energy(solver.ctx, U.detach().contiguous(), out, rho0U0sq)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (U,) = ctx.saved_tensors
        g = torch.empty_like(U)
        dgx.dg_kinetic_energy_grad(ctx.solver.ctx, U.detach().contiguous(), g, ctx.rho0U0sq,
                                   float(grad_out.reshape(-1)[0].item()))
        return g, None, None


def kinetic_energy(solver, U: torch.Tensor, rho0U0sq: float = 1.0) -> torch.Tensor:
    """E_k = sum w J |m|^2/rho / (2 rho0 U0^2 |Omega|), shape (1,); differentiable in U."""
    return _KineticEnergy.apply(U, solver, float(rho0U0sq))
