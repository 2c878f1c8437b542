"""Pins of the oracle's SOR smoother (Gauss-Seidel / SOR of "The choice of
C": x <- x + omega (D + omega L)^{-1} (b - A x), L the couplings to earlier
colours) against a dense triangular solve and against Young's closed form
for the spectral radius of red-black SOR on the model Poisson problem (no GPU).
"""

import math

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W


def _colour_rank(h, l):
    rank = np.empty(h.A[l].shape[0], dtype=int)
    for k, c in enumerate(h.colours[l]):
        rank[c] = k
    return rank


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.5])
@pytest.mark.parametrize("case", ["rbgs", "gs4c"])
def test_sor_step_is_dense_preconditioned_richardson(case, omega):
    """One smoothing step equals x + omega (D + omega L)^{-1} (b - A x) with
    L the part of A coupling each node to nodes of earlier colours (dense
    solve; 5-point red-black and Q1 four-colour)."""
    rng = np.random.default_rng(11)
    g = O.Grid(9, 9)
    if case == "rbgs":
        h = O.hierarchy_5pt(g, 0.3, 1.0, O.Options(smoother="rbgs", sor=omega), levels=2)
    else:
        kx = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        ky = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        h = O.hierarchy_q1(g, kx, ky, O.Options(smoother="gs4c", sor=omega), levels=2)
    A = h.A[0].toarray()
    rank = _colour_rank(h, 0)
    D = np.diag(np.diag(A))
    L = np.where(rank[None, :] < rank[:, None], A, 0.0)
    x = rng.standard_normal(g.n_unknowns)
    b = rng.standard_normal(g.n_unknowns)
    got = O.smooth(h, 0, x, b, 1)
    want = x + omega * np.linalg.solve(D + omega * L, b - A @ x)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def _young_radius(omega, mu):
    """Spectral radius of SOR for a consistently ordered matrix whose Jacobi
    iteration has spectral radius mu (Young's theorem)."""
    w_opt = 2.0 / (1.0 + math.sqrt(1.0 - mu * mu))
    if omega >= w_opt:
        return omega - 1.0
    r = 0.5 * (omega * mu + math.sqrt(omega * omega * mu * mu - 4.0 * (omega - 1.0)))
    return r * r


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.3, 1.6, 1.85])
def test_red_black_sor_radius_is_youngs(omega):
    """The 5-point Laplacian in red-black order is consistently ordered; its
    Jacobi radius is cos(pi h).  The spectral radius of one oracle SOR step
    (b = 0, built column by column from unit vectors) equals Young's value,
    including omega = 1 (cos^2(pi h)) and omega above the optimum (omega - 1)."""
    n = 17
    g = O.Grid(n, n)
    h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs", sor=omega), levels=2)
    m = g.n_unknowns
    M = np.empty((m, m))
    zero = np.zeros(m)
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        M[:, k] = O.smooth(h, 0, e, zero, 1)
    rho = max(abs(np.linalg.eigvals(M)))
    want = _young_radius(omega, math.cos(math.pi * g.hx))
    assert abs(rho - want) <= 2e-6 * max(want, 1e-3), (rho, want)


def test_sor_cycle_converges_and_one_is_gauss_seidel():
    """sor = 1 reproduces the Gauss-Seidel cycle exactly; an over-relaxed
    F-cycle on the model problem still solves to 1e-10."""
    g = O.Grid(33, 33)
    b = g.pack(W.normal_field(33, 33, 2))
    x0 = np.zeros_like(b)
    gs = O.solve(O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs")), b, x0, 1e-10, 50)
    s1 = O.solve(O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs", sor=1.0)), b, x0, 1e-10, 50)
    s15 = O.solve(O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs", sor=1.15)), b, x0, 1e-10, 50)
    assert np.array_equal(gs.x, s1.x)
    assert s15.status == O.OK and s15.cycles <= 15
