"""torch.autograd bindings of the HOPE right-hand side: the forward runs the
library's tendency or Runge-Kutta step, the backward its hand-written
vector-Jacobian product.  States here are interior fields (3, 6, n, n) on the
GPU in float64; the padded buffers the library works on are internal.

``rollout`` differentiates a whole time integration with checkpointing: the
forward keeps every k-th state, the backward recomputes the states of one
segment at a time from its checkpoint and runs the step adjoints in reverse,
so memory grows with steps/k + k states instead of 3 x steps stage states.
"""
from __future__ import annotations

import torch

from .grid import Grid


def _padded(grid: Grid, q: torch.Tensor) -> torch.Tensor:
    qp = grid.new_state(q.device)
    grid.interior(qp).copy_(q)
    return qp


class _Tendency(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, grid):
        ctx.grid = grid
        ctx.save_for_backward(q)
        return grid.tendency(_padded(grid, q))

    @staticmethod
    def backward(ctx, w):
        (q,) = ctx.saved_tensors
        grid = ctx.grid
        return grid.tendency_vjp(_padded(grid, q), w.contiguous()), None


class _RkStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, grid, dt, scheme):
        ctx.grid, ctx.dt, ctx.scheme = grid, dt, scheme
        ctx.save_for_backward(q)
        qp = _padded(grid, q)
        grid.rk_step(qp, dt, scheme)
        return grid.interior(qp).contiguous()

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        grid = ctx.grid
        return grid.rk_step_vjp(_padded(grid, q), ctx.dt, g.contiguous(), ctx.scheme), None, None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q0, grid, dt, steps, every, scheme, check_state):
        ctx.grid, ctx.dt, ctx.steps, ctx.every, ctx.scheme = grid, dt, steps, every, scheme
        qp = _padded(grid, q0)
        ws = grid.workspace()
        checkpoints = []
        for s in range(steps):
            if s % every == 0:
                if check_state and s > 0:
                    _raise_if_bad(grid, qp, s)
                checkpoints.append(grid.interior(qp).clone())
            grid.rk_step(qp, dt, scheme, ws)
        if check_state:
            _raise_if_bad(grid, qp, steps)
        ctx.checkpoints = checkpoints
        return grid.interior(qp).contiguous()

    @staticmethod
    def backward(ctx, g):
        grid, dt, steps, every, scheme = ctx.grid, ctx.dt, ctx.steps, ctx.every, ctx.scheme
        ws = grid.workspace()
        vws = grid.rk_vjp_workspace()
        cot = g.contiguous().clone()
        nxt = torch.empty_like(cot)
        for seg in reversed(range(len(ctx.checkpoints))):
            first = seg * every
            last = min(steps, first + every)
            # states at the start of each step of this segment
            qp = _padded(grid, ctx.checkpoints[seg])
            states = []
            for _ in range(first, last):
                states.append(qp.clone())
                grid.rk_step(qp, dt, scheme, ws)
            del qp
            for qs in reversed(states):
                grid.rk_step_vjp(qs, dt, cot, scheme, out=nxt, ws=vws)
                cot, nxt = nxt, cot
            del states
        ctx.checkpoints = None
        return cot, None, None, None, None, None, None


def _raise_if_bad(grid: Grid, qp: torch.Tensor, step: int):
    bad = grid.bad_cells(qp)
    if bad:
        raise FloatingPointError(f"after step {step}: {bad} cells with a thickness that is not positive "
                                 "or a variable that is not finite")


def tendency(grid: Grid, q: torch.Tensor) -> torch.Tensor:
    """dq/dt of the interior state q (3, 6, n, n), differentiable."""
    return _Tendency.apply(q, grid)


def rk_step(grid: Grid, q: torch.Tensor, dt: float, scheme: str = "ssp3") -> torch.Tensor:
    """One Runge-Kutta step of the interior state q, differentiable."""
    return _RkStep.apply(q, grid, float(dt), scheme)


def rollout(grid: Grid, q0: torch.Tensor, dt: float, steps: int, checkpoint_every: int = 5,
            scheme: str = "ssp3", check_state: bool = False) -> torch.Tensor:
    """The state after ``steps`` Runge-Kutta steps from q0, differentiable with
    checkpoints every ``checkpoint_every`` steps.  With ``check_state`` the
    state is checked at every checkpoint and at the end, and a thickness that
    is not positive or a variable that is not finite raises
    FloatingPointError naming the step (each check waits for the stream)."""
    if steps < 1 or checkpoint_every < 1:
        raise ValueError("steps and checkpoint_every must be positive")
    return _Rollout.apply(q0, grid, float(dt), int(steps), int(checkpoint_every), scheme, bool(check_state))
