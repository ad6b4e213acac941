"""torch.autograd wrapper: ensemble solve forward, discrete adjoint backward.

``solve_ad(spec, y0, theta)`` returns (y_out, y_final) as differentiable
functions of the initial conditions y0 [d][n] and the parameters theta ([p]
shared by all trajectories, or [p][n]).  Backward runs gs_solve_vjp on the
tape of the forward call: the exact derivative of the discrete solution with
the accepted steps held fixed (the transpose of eq:stage-sens).  For shared
parameters the per-trajectory cotangents are summed over the ensemble
(eq:chain).  Everything numerical runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import api


@dataclass
class SolveSpec:
    """Non-differentiable part of an ensemble problem."""
    rhs: str | int
    tableau: str | int
    t0: object
    t1: object
    rtol: object
    atol: object
    t_out: object = None
    # 0: store mode (every accepted step on the tape, no replay in the
    # backward pass, the fastest measured) when that tape fits in half the
    # free device memory, else checkpoints every 32 accepted steps
    ckpt_every: int = 0
    ckpt_capacity: int = 0          # 0: sized from the steps of earlier calls, grown on overflow
    launch: api.Launch = field(default_factory=api.Launch)
    last_solution: object = None    # the Solution of the latest forward
    steps_seen: int = 0             # most accepted steps of any trajectory so far


def _tape_mode(prob: api.Problem, spec: SolveSpec, steps: int) -> tuple[int, int]:
    """(ckpt_every, ckpt_capacity) for a forward expected to take up to
    `steps` accepted steps per trajectory."""
    k = spec.ckpt_every
    if k == 0:
        k = 1
        free = torch.cuda.mem_get_info(prob.y0.device)[0]
        L = api.Launch(**{**spec.launch.__dict__, "ckpt_every": 1, "ckpt_capacity": steps + 2})
        if api.workspace_bytes(prob, L) > free // 2:
            k = 32
    return k, (spec.ckpt_capacity or steps // k + 2)


def _solve_with_tape(prob: api.Problem, spec: SolveSpec) -> api.Solution:
    """Forward with a tape.  The capacity comes from the most steps seen in
    earlier calls (with a quarter in hand); only a trajectory that overflows
    it makes the forward run again, once, with the capacity it needs."""
    steps = spec.steps_seen + spec.steps_seen // 4 if spec.steps_seen else 256
    while True:
        k, cap = _tape_mode(prob, spec, steps)
        L = api.Launch(**{**spec.launch.__dict__, "ckpt_every": k, "ckpt_capacity": cap})
        sol = api.solve(prob, L)
        nmax = int(sol.n_accepted.max())
        spec.steps_seen = max(spec.steps_seen, nmax)
        if spec.ckpt_capacity or nmax // k + 2 <= cap:
            return sol
        steps = nmax


class GsSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, theta, spec: SolveSpec):
        prob = api.make_problem(spec.rhs, spec.tableau, y0.detach(), theta.detach(), spec.t0,
                                spec.t1, spec.rtol, spec.atol, spec.t_out, device=y0.device)
        sol = _solve_with_tape(prob, spec)
        spec.last_solution = sol
        ctx.sol = sol
        ctx.shared_theta = theta.dim() == 1
        ctx.mark_non_differentiable(sol.status)
        if sol.y_out is not None:
            y_out = sol.y_out
        else:
            y_out = y0.new_zeros((0, prob.n, prob.d) if sol.launch.out_layout == "knd"
                                 else (prob.d, 0, prob.n))
        return y_out, sol.y_final, sol.status

    @staticmethod
    def backward(ctx, g_out, g_final, _g_status):
        sol = ctx.sol
        yo = None
        if sol.y_out is not None and g_out is not None:
            if sol.launch.out_layout == "knd":  # y_out [K][n][d]; cotangents go in [d][K][n]
                g_out = g_out.permute(2, 0, 1)
            yo = g_out.contiguous().unsqueeze(0)
        yf = None if g_final is None else g_final.contiguous().unsqueeze(0)
        if yo is None and yf is None:
            return None, None, None
        # the adjoint in the forward's launch shape (as tune_gradient times it)
        y0bar, thbar = api.solve_vjp(sol, ybar_final=yf, ybar_out=yo, block=sol.launch.block,
                                     grid=sol.launch.grid)
        thbar = thbar[0]
        if ctx.shared_theta:
            thbar = thbar.sum(dim=1)
        return y0bar[0], thbar, None


def solve_ad(spec: SolveSpec, y0: torch.Tensor, theta: torch.Tensor):
    """Differentiable ensemble solve: returns (y_out [d][K][n], y_final [d][n],
    status [n])."""
    return GsSolveFn.apply(y0, theta, spec)
