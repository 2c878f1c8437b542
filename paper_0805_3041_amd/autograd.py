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


def _forward(solver: mg.Solver, f: torch.Tensor, tol: float, max_cycles: int) -> torch.Tensor:
    u = torch.zeros_like(f)
    info = solver.solve(f.detach().contiguous(), u, tol, max_cycles, history=False)
    if info.status != mg.MG_OK:
        raise RuntimeError(f"forward solve did not converge: {mg.status_string(info.status)}, "
                           f"rel_res {info.rel_res:.3e} after {info.cycles} cycles")
    return u


def _adjoint(solver: mg.Solver, u: torch.Tensor, gu: torch.Tensor, tol: float, max_cycles: int):
    lam = torch.zeros_like(u)
    info = solver.solve(gu.detach().contiguous(), lam, tol, max_cycles, history=False)
    if info.status != mg.MG_OK:
        raise RuntimeError(f"adjoint solve did not converge: {mg.status_string(info.status)}")
    return solver.coeff_grad(u, lam), lam


class MGSolve(torch.autograd.Function):
    """u = MGSolve.apply(a, f, tol, max_cycles, opts).

    a: float64 cuda tensor [ny-1][nx-1] (cells, > 0); f: float64 cuda tensor
    [ny][nx] (nodes).  opts: dict of mg.Solver options (smoother, nu_pre, ...).
    A handle is set up for the call and destroyed by its backward.
    """

    @staticmethod
    def forward(ctx, a: torch.Tensor, f: torch.Tensor, tol: float = 1e-12, max_cycles: int = 500,
                opts: dict | None = None):
        opts = dict(opts or {})
        opts.setdefault("smoother", "gs4c")
        ny, nx = f.shape
        solver = mg.Solver(nx, ny, kx=a.detach().contiguous(), **opts)
        try:
            u = _forward(solver, f, tol, max_cycles)
        except RuntimeError:
            solver.close()
            raise
        ctx.solver = solver
        ctx.tol, ctx.max_cycles = tol, max_cycles
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu: torch.Tensor):
        (u,) = ctx.saved_tensors
        try:
            da, lam = _adjoint(ctx.solver, u, gu, ctx.tol, ctx.max_cycles)
        finally:
            ctx.solver.close()
            ctx.solver = None
        return da, lam, None, None, None


def solve(a: torch.Tensor, f: torch.Tensor, tol: float = 1e-12, max_cycles: int = 500, **opts) -> torch.Tensor:
    """Differentiable u(a, f); see MGSolve."""
    return MGSolve.apply(a, f, tol, max_cycles, opts)


class _ReusedSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a: torch.Tensor, f: torch.Tensor, owner: "GradientSolver"):
        solver = owner._prepare(a.detach().contiguous())
        u = _forward(solver, f, owner.tol, owner.max_cycles)
        ctx.owner, ctx.generation = owner, owner.generation
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu: torch.Tensor):
        (u,) = ctx.saved_tensors
        owner = ctx.owner
        if owner.solver is None or owner.generation != ctx.generation:
            raise RuntimeError("GradientSolver: a later call replaced the operators (or close() ran) before this "
                               "backward; run each call's backward before the next call")
        da, lam = _adjoint(owner.solver, u, gu, owner.tol, owner.max_cycles)
        return da, lam, None


class GradientSolver:
    """Differentiable u(a, f) on one grid, keeping one handle across calls.

    The first call sets the handle up for its a; every later call rebuilds
    the operators for the new a in the handle's device buffers
    (mg_update_coeffs, no allocation), the usual case in a gradient loop
    where a changes every step.  Forward and backward are those of MGSolve.
    Calls are sequential: a call's backward must run before the next call
    (which replaces the operators); a backward that finds them replaced
    raises.  close() destroys the handle.
    """

    def __init__(self, nx: int, ny: int, tol: float = 1e-12, max_cycles: int = 500, **opts):
        self.nx, self.ny, self.tol, self.max_cycles = nx, ny, tol, max_cycles
        self.opts = dict(opts)
        self.opts.setdefault("smoother", "gs4c")
        self.solver: mg.Solver | None = None
        self.generation = 0

    def _prepare(self, a: torch.Tensor) -> mg.Solver:
        if self.solver is None:
            self.solver = mg.Solver(self.nx, self.ny, kx=a, **self.opts)
        else:
            self.solver.update_coefficients(a)
        self.generation += 1
        return self.solver

    def __call__(self, a: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
        if tuple(f.shape) != (self.ny, self.nx):
            raise ValueError(f"f must have shape {(self.ny, self.nx)}, got {tuple(f.shape)}")
        return _ReusedSolve.apply(a, f, self)

    def close(self) -> None:
        if self.solver is not None:
            self.solver.close()
            self.solver = None
        self.generation += 1

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
