"""Refined (graded) tensor grids, the anisotropically refined grids of the
"Anisotropies" section (refinement toward one side as in "Different
coordinate systems"): the library folds the cell widths into the Q1 cell
coefficients at setup and runs the cell-coefficient kernels; per cycle to
1e-12 against the oracle's element-by-element assembly on the refined grid
(coarse levels Galerkin), for 1-D and 2-D coefficients, x and y refinement,
fused, per-op, interpreter and line-smoother paths; second-order
convergence of the GPU solution; coefficient updates; rejected uses."""

import ctypes

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W
from tests.problems import Problem
from tests.test_gpu_parity import check_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mg():
    from paper_0805_3041_amd import mg
    return mg


CASES = [
    dict(p=dict(nx=129, ny=129, q1="unit", smoother="gs4c", grade=(2.0, 0.0)), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c", grade=(2.0, -1.5)), cta=300),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c", grade=(2.0, 0.0)), cta=300),
    dict(p=dict(nx=65, ny=65, q1="unit", smoother="jacobi", grade=(3.0, 1.0)), cta=0),
    dict(p=dict(nx=257, ny=257, q1="sphere", smoother="gs4c", grade=(1.5, 0.0)), cta=300),
    dict(p=dict(nx=97, ny=49, q1="unit", smoother="gs4c", grade=(1.0, 2.0)), cta=100, extra=dict(tile_mode="per_op")),
    dict(p=dict(nx=65, ny=65, q1="unit", smoother="gstri_x", grade=(3.0, 0.0)), cta=0),
    dict(p=dict(nx=129, ny=129, q1="unit", smoother="gsadi", grade=(2.0, 2.0)), cta=300),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c", grade=(-2.0, 0.0)), cta=300,
         extra=dict(tile_mode="wide")),
]


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_graded_per_cycle(case):
    p = Problem(**case["p"])
    check_parity(p, p.rhs(2), W.uniform_field(p.nx, p.ny, 1, p.periodic_y), 3, coarse_cta_nodes=case["cta"],
                 **case.get("extra", {}))


def test_graded_manufactured_second_order_on_gpu():
    """u = sin(pi x) sin(pi y) with the lumped right-hand side on grids refined
    toward x = 0 and toward y = 1: the GPU solution's nodal max error falls by
    4 +- 0.2 from 257^2 to 513^2 to 1025^2."""
    mg = _mg()
    errs = []
    for n in (257, 513, 1025):
        xs, ys = W.graded_nodes(n, 2.0), W.graded_nodes(n, -1.5)
        X, Y = np.meshgrid(xs, ys)
        u = np.sin(np.pi * X) * np.sin(np.pi * Y)
        b = torch.tensor(W.lumped_rhs(2 * np.pi**2 * u, xs, ys), device="cuda")
        one = torch.ones((n - 1, n - 1), dtype=torch.float64, device="cuda")
        s = mg.Solver(n, n, kx=one, ky=one, xs=xs, ys=ys, smoother="gs4c")
        try:
            x = torch.zeros_like(b)
            info = s.solve(b, x, 1e-10, 200, history=False)
        finally:
            s.close()
        assert info.status == mg.MG_OK
        errs.append(np.abs(x.cpu().numpy() - u).max())
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(abs(q - 4.0) < 0.2 for q in ratios), (errs, ratios)


def test_graded_update_equals_fresh_setup():
    """mg_update_coeffs on a refined-grid handle folds the new cells with the
    same widths: the next solve equals a fresh setup's bit for bit."""
    mg = _mg()
    n = 129
    xs, ys = W.graded_nodes(n, 2.0), W.graded_nodes(n, 1.0)
    a1 = torch.tensor(np.exp(W.gaussian_random_field(n - 1, 5)), device="cuda")
    a2 = torch.tensor(np.exp(0.5 * W.gaussian_random_field(n - 1, 6)), device="cuda")
    rhs = torch.tensor(W.normal_field(n, n, 3), device="cuda")
    s = mg.Solver(n, n, kx=a1, ky=a1, xs=xs, ys=ys, smoother="gs4c", coarse_cta_nodes=300)
    f = mg.Solver(n, n, kx=a2, ky=a2, xs=xs, ys=ys, smoother="gs4c", coarse_cta_nodes=300)
    try:
        s.update_coefficients(a2)
        xa, xb = torch.zeros_like(rhs), torch.zeros_like(rhs)
        s.solve(rhs, xa, 1e-300, 3, history=False)
        f.solve(rhs, xb, 1e-300, 3, history=False)
    finally:
        s.close()
        f.close()
    assert torch.equal(xa, xb)


def test_graded_unsupported_entry_points():
    mg = _mg()
    n = 33
    xs = W.graded_nodes(n, 2.0)
    a = torch.ones((n - 1, n - 1), dtype=torch.float64, device="cuda")
    s = mg.Solver(n, n, kx=a, ky=a, xs=xs, smoother="gs4c")
    try:
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        with pytest.raises(mg.MGError) as e:
            s.coeff_grad(u, u)
        assert e.value.status == mg.MG_EUNSUPPORTED
        with pytest.raises(mg.MGError) as e:
            mg.mg_residual_noalloc(s.grid, s.coeffs, u, u)
        assert e.value.status == mg.MG_EUNSUPPORTED
    finally:
        s.close()
