"""Differentiable solve of the variable-coefficient problem -div(a grad u) = f.

``MGSolve.apply(a, f)`` returns u = A(a)^{-1} f computed by the library's
F-cycle (Q1 operator with per-cell coefficient a, lumped right-hand side
b = f).  Its backward pass is the adjoint of the discrete solve: with
g = dL/du, it solves A^T lam = g (A is symmetric, so the same hierarchy and
the same F-cycle serve) and returns

    dL/da_c = -lam_e^T K_c u_e   (per cell, library kernel mg_coeff_grad)
    dL/df   = lam.

This is the gradient of the converged discrete solution, independent of the
cycle's iterates, so both solves are run to a tight tolerance.
"""

from __future__ import annotations

import torch

from . import mg


class MGSolve(torch.autograd.Function):
    """u = MGSolve.apply(a, f, tol, max_cycles, opts).

    a: float64 cuda tensor [ny-1][nx-1] (cells, > 0); f: float64 cuda tensor
    [ny][nx] (nodes).  opts: dict of mg.Solver options (smoother, nu_pre, ...).
    """

    @staticmethod
    def forward(ctx, a: torch.Tensor, f: torch.Tensor, tol: float = 1e-12, max_cycles: int = 500,
                opts: dict | None = None):
        opts = dict(opts or {})
        opts.setdefault("smoother", "gs4c")
        ny, nx = f.shape
        a_d = a.detach().contiguous()
        solver = mg.Solver(nx, ny, kx=a_d, ky=a_d, **opts)
        u = torch.zeros_like(f)
        info = solver.solve(f.detach().contiguous(), u, tol, max_cycles, history=False)
        if info.status != mg.MG_OK:
            solver.close()
            raise RuntimeError(f"forward solve did not converge: {mg.status_string(info.status)}, "
                               f"rel_res {info.rel_res:.3e} after {info.cycles} cycles")
        ctx.solver = solver
        ctx.tol, ctx.max_cycles = tol, max_cycles
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu: torch.Tensor):
        (u,) = ctx.saved_tensors
        solver = ctx.solver
        try:
            lam = torch.zeros_like(u)
            info = solver.solve(gu.detach().contiguous(), lam, ctx.tol, ctx.max_cycles, history=False)
            if info.status not in (mg.MG_OK,):
                raise RuntimeError(f"adjoint solve did not converge: {mg.status_string(info.status)}")
            da = solver.coeff_grad(u, lam)
        finally:
            solver.close()
            ctx.solver = None
        return da, lam, None, None, None


def solve(a: torch.Tensor, f: torch.Tensor, tol: float = 1e-12, max_cycles: int = 500, **opts) -> torch.Tensor:
    """Differentiable u(a, f); see MGSolve."""
    return MGSolve.apply(a, f, tol, max_cycles, opts)
