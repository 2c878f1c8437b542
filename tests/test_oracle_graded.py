"""Pins of the oracle's Q1 operator on refined (graded) tensor grids, the
anisotropically refined grids of the "Anisotropies" section: against the
equidistant assembly, a brute-force quadrature of the bilinear basis on each
rectangle, and second-order nodal convergence of a manufactured solution
under smooth grading (no GPU)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mg_oracle as O
import workloads as W


def test_graded_assembly_on_an_equidistant_grid_is_the_plain_one():
    g = O.Grid(9, 7)
    rng = np.random.default_rng(31)
    kx, ky = rng.uniform(0.5, 2.0, (2, g.ncy, g.ncx))
    A = O.assemble_q1_graded(g, np.linspace(0, 1, 9), np.linspace(0, 1, 7), kx, ky).toarray()
    B = O.assemble_q1(g, kx, ky).toarray()
    np.testing.assert_allclose(A, B, rtol=0, atol=1e-12 * np.abs(B).max())


def _bilinear_quadrature_matrix(xs, ys, kx, ky):
    """Dense stiffness matrix over every stored node by 2x2 Gauss quadrature
    of kx phi_p,x phi_q,x + ky phi_p,y phi_q,y on each rectangle, with the
    bilinear basis written out (exact: the integrand is at most quadratic in
    each variable)."""
    nx, ny = len(xs), len(ys)
    K = np.zeros((nx * ny, nx * ny))
    gp = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    for cj in range(ny - 1):
        y0, y1 = ys[cj], ys[cj + 1]
        for ci in range(nx - 1):
            x0, x1 = xs[ci], xs[ci + 1]
            hx, hy = x1 - x0, y1 - y0
            nodes = [(cj + b, ci + a) for b in range(2) for a in range(2)]
            for sx in gp:
                for sy in gp:
                    x = x0 + 0.5 * (sx + 1) * hx
                    y = y0 + 0.5 * (sy + 1) * hy
                    wq = 0.25 * hx * hy  # Gauss weights 1 x 1 on [-1, 1]^2, Jacobian hx hy / 4
                    lx = [(x1 - x) / hx, (x - x0) / hx]
                    ly = [(y1 - y) / hy, (y - y0) / hy]
                    dlx = [-1.0 / hx, 1.0 / hx]
                    dly = [-1.0 / hy, 1.0 / hy]
                    gx = [dlx[a] * ly[b] for b in range(2) for a in range(2)]
                    gy = [lx[a] * dly[b] for b in range(2) for a in range(2)]
                    for p, (jp, ip) in enumerate(nodes):
                        for q, (jq, iq) in enumerate(nodes):
                            K[jp * nx + ip, jq * nx + iq] += wq * (kx[cj, ci] * gx[p] * gx[q]
                                                                   + ky[cj, ci] * gy[p] * gy[q])
    return K


def test_graded_assembly_equals_brute_force_quadrature():
    nx, ny = 9, 7
    g = O.Grid(nx, ny)
    xs = W.graded_nodes(nx, 2.5)
    ys = W.graded_nodes(ny, -1.2)
    rng = np.random.default_rng(32)
    kx, ky = rng.uniform(0.5, 2.0, (2, g.ncy, g.ncx))
    K = _bilinear_quadrature_matrix(xs, ys, kx, ky)
    interior = [j * nx + i for j in g.uy for i in g.ux]
    ref = K[np.ix_(interior, interior)] / ((1.0 / (nx - 1)) * (1.0 / (ny - 1)))
    A = O.assemble_q1_graded(g, xs, ys, kx, ky).toarray()
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(A, A.T, atol=1e-14 * np.abs(A).max())


@pytest.mark.parametrize("ax,ay", [(2.0, 0.0), (2.0, -1.5), (3.0, 1.0)])
def test_graded_manufactured_second_order(ax, ay):
    """u = sin(pi x) sin(pi y), f = 2 pi^2 u, lumped right-hand side on grids
    refined toward x = 0 (and toward one y side): the nodal max error falls by
    4 +- 0.2 per halving of the spacing (33, 65, 129 nodes)."""
    errs = []
    for n in (33, 65, 129):
        g = O.Grid(n, n)
        xs, ys = W.graded_nodes(n, ax), W.graded_nodes(n, ay)
        X, Y = np.meshgrid(xs, ys)
        u = np.sin(np.pi * X) * np.sin(np.pi * Y)
        b = W.lumped_rhs(2 * np.pi**2 * u, xs, ys)
        ones = np.ones((n - 1, n - 1))
        x = spla.spsolve(O.assemble_q1_graded(g, xs, ys, ones, ones).tocsc(), g.pack(b))
        errs.append(np.abs(x - g.pack(u)).max())
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(abs(q - 4.0) < 0.2 for q in ratios), (errs, ratios)


def test_graded_nodes_refine_toward_one_side():
    x = W.graded_nodes(65, 2.0)
    h = np.diff(x)
    assert x[0] == 0.0 and x[-1] == 1.0 and np.all(h > 0) and np.all(np.diff(h) > 0)
    assert abs(h[-1] / h[0] - np.exp(2.0 * 63 / 64)) < 1e-9 * np.exp(2.0)


def test_graded_x_on_a_periodic_grid_equals_elementwise_cells():
    """Refinement along x of a periodic-y grid: the same matrix as the plain
    assembly with the refinement folded into the cells by hand (the x part
    scaled by hy0/hx_c / (hy0/hx0), the y part by hx_c/hx0)."""
    g = O.Grid(9, 8, periodic_y=True)
    xs = W.graded_nodes(9, 2.0)
    rng = np.random.default_rng(33)
    kx, ky = rng.uniform(0.5, 2.0, (2, g.ncy, g.ncx))
    r = np.diff(xs) / g.hx
    A = O.assemble_q1_graded(g, xs, None, kx, ky).toarray()
    B = O.assemble_q1(g, kx / r[None, :], ky * r[None, :]).toarray()
    np.testing.assert_allclose(A, B, rtol=0, atol=1e-12 * np.abs(B).max())
