"""Adjoint gradient of the Q1 solve (dL/da per cell, dL/df) through the
library against the oracle's direct-solve adjoint and central differences."""

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mods():
    from paper_0805_3041_amd import autograd as AG
    from paper_0805_3041_amd import mg
    return mg, AG


def _problem(n, seed=5):
    a = np.exp(W.gaussian_random_field(n - 1, seed))
    f, ustar = W.manufactured_sine(n)
    return a, f, ustar


def _loss(u, ustar):
    d = u - ustar
    return 0.5 * torch.sum(d * d)


@pytest.mark.parametrize("periodic", [False, True])
def test_coeff_grad_kernel_matches_oracle(periodic):
    mg, _ = _mods()
    nx, ny = (33, 32) if periodic else (33, 33)
    g = O.Grid(nx, ny, periodic)
    rng = np.random.default_rng(31)
    u = W.zero_boundary(rng.standard_normal((ny, nx)), periodic)
    lam = W.zero_boundary(rng.standard_normal((ny, nx)), periodic)
    ncy = ny if periodic else ny - 1
    a = torch.ones((ncy, nx - 1), dtype=torch.float64, device="cuda")
    s = mg.Solver(nx, ny, periodic_y=periodic, kx=a, smoother="gs4c")
    got = s.coeff_grad(torch.tensor(u, device="cuda"), torch.tensor(lam, device="cuda")).cpu().numpy()
    s.close()
    ref = O.q1_coeff_grad(g, u, lam, "a")
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_gradient_matches_oracle_direct_adjoint():
    """dL/da and dL/df from the F-cycle adjoint equal the oracle's direct-solve adjoint to 1e-10."""
    mg, AG = _mods()
    n = 33
    a, f, ustar = _problem(n)
    ustar = 1.3 * ustar
    g = O.Grid(n, n)
    _, lam_o, da_o, _ = O.adjoint_gradient(g, a, f, ustar)
    at = torch.tensor(a, device="cuda", requires_grad=True)
    ft = torch.tensor(f, device="cuda", requires_grad=True)
    u = AG.solve(at, ft, tol=1e-13, max_cycles=200)
    _loss(u, torch.tensor(ustar, device="cuda")).backward()
    da = at.grad.cpu().numpy()
    df = ft.grad.cpu().numpy()
    assert np.linalg.norm(da - da_o) <= 1e-10 * np.linalg.norm(da_o)
    assert np.linalg.norm(df - lam_o) <= 1e-10 * np.linalg.norm(lam_o)


def test_gradient_central_differences_full():
    """Every component of dL/da against central differences of L (GPU forward solves), <= 1e-5 relative."""
    mg, AG = _mods()
    n = 17
    a, f, ustar = _problem(n, seed=6)
    us = torch.tensor(1.5 * ustar, device="cuda")
    ft = torch.tensor(f, device="cuda")
    at = torch.tensor(a, device="cuda", requires_grad=True)
    _loss(AG.solve(at, ft, tol=1e-13), us).backward()
    grad = at.grad.cpu().numpy()

    def L(aa):
        with torch.no_grad():
            return _loss(AG.solve(torch.tensor(aa, device="cuda"), ft, tol=1e-13), us).item()

    tau = 1e-4 * np.abs(a).max()
    fd = np.zeros_like(a)
    for idx in np.ndindex(a.shape):
        ap, am = a.copy(), a.copy()
        ap[idx] += tau
        am[idx] -= tau
        fd[idx] = (L(ap) - L(am)) / (2 * tau)
    assert np.linalg.norm(grad - fd) <= 1e-5 * np.linalg.norm(fd)


@pytest.mark.slow
def test_grf2049_directional_derivative_and_tangent_linear():
    """Full size (2049^2 nodes, 2048^2 cells, a = exp(GRF)): directional central
    difference and the tangent-linear value -(u - u*)^T A^{-1} (dA u) (dA u from
    the library's residual of a solver with coefficient da) agree with
    <dL/da, da> to 1e-5."""
    mg, AG = _mods()
    n = 2049
    a, f, ustar = W.grf_problem(n, 5)
    us = torch.tensor(ustar, device="cuda")
    ft = torch.tensor(f, device="cuda")
    at = torch.tensor(a, device="cuda", requires_grad=True)
    # FP64 evaluation of b - A x at h = 1/2048 with coefficients up to e^4 has a
    # relative floor near 1e-10 for this smooth right-hand side: solve to 3e-10
    tol = 3e-10
    u = AG.solve(at, ft, tol=tol, max_cycles=300)
    _loss(u, us).backward()
    grad = at.grad
    rng = np.random.default_rng(41)
    # a relative perturbation direction (a spans ~3 decades): da = a * U[0.5, 1.5]
    da = torch.tensor(a * rng.uniform(0.5, 1.5, a.shape), device="cuda")
    lin = torch.sum(grad * da).item()
    # central-difference truncation ~ tau^2 (relative perturbation of a); 2e-4
    # keeps it near 1e-7 while L(a +- tau da) still differ by ~4e-4 |L'|
    tau = 2e-4
    with torch.no_grad():
        lp = _loss(AG.solve(at.detach() + tau * da, ft, tol=tol, max_cycles=300), us).item()
        lm = _loss(AG.solve(at.detach() - tau * da, ft, tol=tol, max_cycles=300), us).item()
    fd = (lp - lm) / (2 * tau)
    assert abs(fd - lin) <= 1e-5 * abs(lin), (fd, lin)
    # tangent linear: du = -A^{-1} (dA u); dA u = -(0 - A(da) u) from mg_residual
    s_da = mg.Solver(n, n, kx=da, smoother="gs4c")
    r = torch.zeros_like(u)
    s_da.residual(torch.zeros_like(u), u.detach().contiguous(), r)
    s_da.close()
    dAu = -r
    s = mg.Solver(n, n, kx=at.detach(), smoother="gs4c")
    du = torch.zeros_like(u)
    info = s.solve(-dAu, du, tol, 300)
    s.close()
    assert info.status == 0
    tl = torch.sum((u.detach() - us) * du).item()
    assert abs(tl - lin) <= 1e-5 * abs(lin), (tl, lin)
