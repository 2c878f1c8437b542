"""Pins of the spherical-coordinate coefficients ("Different coordinate
systems": the operator's coefficients carry the factor r^2 sin(theta)) and of
the oracle's Q1 operator on them (no GPU)."""

import numpy as np
import scipy.sparse.linalg as spla

from oracle import mg_oracle as O
import workloads as W


def test_sphere_coefficients_are_the_weighted_metric():
    """kx / ky = r^2 (Lt / Lr)^2 and ky / sin(theta) = Lr / Lt at every cell
    midpoint (the weak form's r^2 sin(theta) weight and the mapping)."""
    nx, ny = 9, 17
    kx, ky = W.sphere_cell_coefficients(nx, ny)
    assert kx.shape == (ny - 1, nx - 1) and ky.shape == (ny - 1, nx - 1)
    lr, lt = W.SPHERE_R1 - W.SPHERE_R0, W.SPHERE_T1 - W.SPHERE_T0
    r = W.SPHERE_R0 + lr * (np.arange(nx - 1) + 0.5) / (nx - 1)
    t = W.SPHERE_T0 + lt * (np.arange(ny - 1) + 0.5) / (ny - 1)
    np.testing.assert_allclose(kx / ky, np.broadcast_to(r[None, :] ** 2 * (lt / lr) ** 2, kx.shape), rtol=1e-14)
    np.testing.assert_allclose(ky, np.broadcast_to(np.sin(t)[:, None] * lr / lt, ky.shape), rtol=1e-14)


def test_sphere_discretisation_is_second_order():
    """The Q1 operator with the midpoint cell coefficients, solved directly
    for the manufactured u = sin(pi xi) sin(pi eta), has a max-norm error
    that falls by 4 per halving of h."""
    errs = []
    for n in (17, 33, 65):
        g = O.Grid(n, n)
        kx, ky = W.sphere_cell_coefficients(n, n)
        A = O.assemble_q1(g, kx, ky)
        f, u = W.sphere_manufactured(n)
        uh = spla.spsolve(A.tocsc(), g.pack(f))
        errs.append(np.abs(uh - g.pack(u)).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.6 < q < 4.4 for q in ratios), (errs, ratios)


def test_sphere_line_smoothing_along_the_strong_direction():
    """Here kx / ky is 6-25 (coupling strongest along r = x): Gauss-Seidel
    over x lines and GSADI solve to 1e-10 in a handful of F-cycles, point
    four-colour GS and y lines need five times as many, the dependence on
    the line direction the paper reports for spherical coordinates."""
    n = 65
    g = O.Grid(n, n)
    kx, ky = W.sphere_cell_coefficients(n, n)
    b = g.pack(W.normal_field(n, n, 3))
    cyc = {}
    for sm in ("gs4c", "gstri_x", "gstri_y", "gsadi"):
        h = O.hierarchy_q1(g, kx, ky, O.Options(smoother=sm))
        r = O.solve(h, b, np.zeros_like(b), 1e-10, 100)
        assert r.status == O.OK, sm
        cyc[sm] = r.cycles
    assert cyc["gstri_x"] <= 8 and cyc["gsadi"] <= 8
    assert cyc["gs4c"] >= 4 * cyc["gstri_x"] and cyc["gstri_y"] >= 4 * cyc["gstri_x"]
