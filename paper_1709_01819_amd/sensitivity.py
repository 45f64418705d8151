"""Steady wall objectives as differentiable functions of theta = (lid speed, wall
temperature, Kn): the forward pass converges the implicit scheme, the backward pass runs the
adjoint iteration (both on the GPU through the C ABI)."""
import torch

from .solver import Solver

LID_SIDE = 3


def config_at(cfg, theta):
    """Copy of a configuration with theta = (lid speed, common wall temperature, Kn)."""
    c = dict(cfg)
    c["wall_u"], c["wall_T"] = list(cfg["wall_u"]), list(cfg["wall_T"])
    c["wall_u"][LID_SIDE] = float(theta[0])
    for s in range(4):
        if cfg["bc"][s] == 0:
            c["wall_T"][s] = float(theta[1])
    c["Kn"] = float(theta[2])
    return c


class SteadyObjective(torch.autograd.Function):
    """J(theta) at the steady state; backward gives dJ/dtheta from one adjoint solve.

    apply(theta, cfg, which, tol, max_iter, adj_tol): theta is a float64 tensor of 3.  The
    forward pass converges the scheme and evaluates J only; the converged solver is kept
    for the backward pass, which runs the adjoint iteration when a gradient is asked for."""

    @staticmethod
    def forward(ctx, theta, cfg, which, tol=1e-12, max_iter=20000, adj_tol=1e-11):
        s = Solver(config_at(cfg, theta.detach().cpu().tolist()))
        it, res, ok = s.solve(tol, max_iter)
        if not ok:
            raise RuntimeError(f"forward solve did not converge ({it} iterations, residual {res})")
        J, _, _ = s.objective(which)
        ctx.solver, ctx.which, ctx.adj_tol, ctx.adj_iter = s, which, adj_tol, 20 * max_iter
        ctx.dtype = theta.dtype
        return torch.as_tensor(J, dtype=theta.dtype)

    @staticmethod
    def backward(ctx, gout):
        s = ctx.solver
        ctx.solver = None  # the adjoint runs once per forward
        grad = None
        if ctx.needs_input_grad[0]:
            _, g, _, _, _ = s.adjoint(ctx.which, ctx.adj_tol, ctx.adj_iter)
            grad = gout * torch.as_tensor(g, dtype=ctx.dtype)
        return grad, None, None, None, None, None
