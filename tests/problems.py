"""Problem descriptions shared by the GPU tests: each builds the oracle's
hierarchy and the library's solver for the same seeded inputs."""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import mg_oracle as O
import workloads as W


@dataclass
class Problem:
    nx: int
    ny: int
    periodic_y: bool = False
    eps: float = 1.0
    q1: str | None = None        # None (5-point), "annulus", "grf", "sphere"
    smoother: str = "rbgs"
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    sor: float = 1.0
    cycle: str = "F"
    levels: int = 0
    coarse_op: str = "default"   # "galerkin": 5-point problems take R A P on the coarse levels
    adaptive_omega: bool = False  # energy-minimising coarse-correction weight
    grade: tuple | None = None    # (ax, ay): refined grid, W.graded_nodes exponents along x and y

    def coords(self):
        """Node coordinates (xs, ys) of a refined grid, or (None, None)."""
        if self.grade is None:
            return None, None
        ax, ay = self.grade
        xs = W.graded_nodes(self.nx, ax) if ax else None
        ys = W.graded_nodes(self.ny, ay) if ay else None
        return xs, ys

    def grid(self):
        return O.Grid(self.nx, self.ny, self.periodic_y)

    def coefficients(self):
        """Cell coefficients (kx, ky, one_d) or None."""
        if self.q1 == "annulus":
            kx, ky = W.annulus_cell_coefficients(self.nx)
            return kx, ky, True
        if self.q1 == "sphere":
            kx, ky = W.sphere_cell_coefficients(self.nx, self.ny)
            return kx, ky, False
        if self.q1 == "grf":
            ncy = self.ny if self.periodic_y else self.ny - 1
            assert ncy == self.nx - 1
            a = np.exp(W.gaussian_random_field(self.nx - 1, 5))
            return a, a, False
        if self.q1 == "unit":
            ncy = self.ny if self.periodic_y else self.ny - 1
            one = np.ones((ncy, self.nx - 1))
            return one, one, False
        return None

    def oracle(self):
        g = self.grid()
        opts = O.Options(cycle=self.cycle, smoother=self.smoother, nu_pre=self.nu_pre, nu_post=self.nu_post,
                         omega=self.omega, sor=self.sor, adaptive_omega=self.adaptive_omega)
        c = self.coefficients()
        if c is None:
            return O.hierarchy_5pt(g, self.eps, 1.0, opts, self.levels, galerkin=self.coarse_op == "galerkin")
        kx, ky, oned = c
        xs, ys = self.coords()
        if xs is not None or ys is not None:
            if oned:
                kx, ky = np.broadcast_to(kx, (g.ncy, g.ncx)), np.broadcast_to(ky, (g.ncy, g.ncx))
            return O.hierarchy_q1(g, kx, ky, opts, self.levels, xs=xs, ys=ys)
        if oned:
            return O.hierarchy_q1(g, kx, ky, opts, self.levels, separable=True)
        return O.hierarchy_q1(g, kx, ky, opts, self.levels)

    def solver(self, precision="fp64", coarse_cta_nodes=0, **extra):
        import torch
        from paper_0805_3041_amd import mg
        c = self.coefficients()
        kw = dict(periodic_y=self.periodic_y, levels=self.levels, cycle=self.cycle, smoother=self.smoother,
                  nu_pre=self.nu_pre, nu_post=self.nu_post, omega=self.omega, sor=self.sor, precision=precision,
                  coarse_cta_nodes=coarse_cta_nodes, coarse_op=self.coarse_op, **extra)
        if self.adaptive_omega:
            kw["adaptive_omega"] = True
        if c is None:
            return mg.Solver(self.nx, self.ny, eps_x=self.eps, eps_y=1.0, **kw)
        kx, ky, oned = c
        dev = "cuda"
        xs, ys = self.coords()
        return mg.Solver(self.nx, self.ny, kx=torch.tensor(kx, device=dev), ky=torch.tensor(ky, device=dev),
                         kx_1d_along_x=oned, xs=xs, ys=ys, **kw)

    def rhs(self, seed=2):
        return W.normal_field(self.nx, self.ny, seed, self.periodic_y)
