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
    ckpt_every: int = 32
    ckpt_capacity: int = 0          # 0: estimate, then grow to fit
    launch: api.Launch = field(default_factory=api.Launch)
    last_solution: object = None    # the Solution of the latest forward


def _solve_with_tape(prob: api.Problem, spec: SolveSpec) -> api.Solution:
    cap = spec.ckpt_capacity or 64
    while True:
        L = api.Launch(**{**spec.launch.__dict__, "ckpt_every": spec.ckpt_every,
                          "ckpt_capacity": cap})
        sol = api.solve(prob, L)
        over = sol.status == 4  # GS_TRAJ_TAPE_OVERFLOW
        if spec.ckpt_capacity or not bool(over.any()):
            return sol
        need = int(sol.n_accepted.max()) // spec.ckpt_every + 2
        cap = max(need, 2 * cap)


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
        y_out = sol.y_out if sol.y_out is not None else y0.new_zeros((prob.d, 0, prob.n))
        return y_out, sol.y_final, sol.status

    @staticmethod
    def backward(ctx, g_out, g_final, _g_status):
        sol = ctx.sol
        yo = None
        if sol.y_out is not None and g_out is not None:
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
