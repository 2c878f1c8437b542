"""Pins of the oracle's line smoothers (TRI, ADI, GSTRI, GSADI of "The choice
of C" and "Smoothing") against closed forms, brute-force constructions and
the method's known behaviour on anisotropic problems (no GPU).
"""

import math

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def sine_mode(g, k, l):
    X, Y = W.node_coords(g.nx, g.ny, g.periodic_y, g.lx, g.ly)
    return g.pack(np.sin(k * np.pi * X / g.lx) * np.sin(l * np.pi * Y / g.ly))


def brute_line_part(g, A, direction):
    """The line part written out with loops over nodes and their two line
    neighbours (tiny grids)."""
    Ad = A.toarray()
    idx = {}
    for jj, j in enumerate(g.uy):
        for ii, i in enumerate(g.ux):
            idx[(i, j)] = jj * len(g.ux) + ii
    T = np.zeros_like(Ad)
    for (i, j), p in idx.items():
        if direction == "x":
            nb = [(i - 1, j), (i, j), (i + 1, j)]
        else:
            jm, jp = j - 1, j + 1
            if g.periodic_y:
                jm, jp = jm % g.ny, jp % g.ny
            nb = [(i, jm), (i, j), (i, jp)]
        for q in nb:
            if q in idx:
                T[p, idx[q]] = Ad[p, idx[q]]
    return T


@pytest.mark.parametrize("direction", ["x", "y"])
@pytest.mark.parametrize("case", ["5pt", "q1", "q1_periodic"])
def test_line_part_equals_brute_force(direction, case):
    """line_part keeps exactly A's couplings of each node with itself and its
    two neighbours along the line (5-point, variable Q1, periodic Q1)."""
    rng = np.random.default_rng(3)
    if case == "5pt":
        g = O.Grid(9, 7)
        A = O.laplace5(g, 0.3, 1.7)
    else:
        g = O.Grid(9, 8, periodic_y=True) if case == "q1_periodic" else O.Grid(9, 7)
        kx = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        ky = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        A = O.assemble_q1(g, kx, ky)
    T = O.line_part(g, A, direction).toarray()
    np.testing.assert_array_equal(T, brute_line_part(g, A, direction))


def green_1d(m, h, eps):
    """Inverse of the Dirichlet second difference eps (-u_{i-1} + 2 u_i - u_{i+1}) / h^2
    on m interior nodes: G_ik = (h^2/eps) min(i,k) (m+1-max(i,k)) / (m+1), 1-based."""
    i = np.arange(1, m + 1)
    I, K = np.meshgrid(i, i, indexing="ij")
    return (h * h / eps) * np.minimum(I, K) * (m + 1 - np.maximum(I, K)) / (m + 1)


def test_tri_x_solves_decoupled_rows_exactly():
    """With eps_y = 0 the 5-point matrix is the x-lines alone: one TRIx step
    with omega = 1 from x = 0 gives each row's 1-D Green's-function solution."""
    g = O.Grid(17, 9)
    eps = 0.7
    A = O.laplace5(g, eps, 0.0)
    T = O.line_part(g, A, "x")
    b = np.random.default_rng(1).standard_normal(g.n_unknowns)
    x = O.tri_step(A, T, np.zeros_like(b), b, 1.0)
    G = green_1d(g.nx - 2, g.hx, eps)
    want = (b.reshape(len(g.uy), -1) @ G.T).reshape(-1)
    np.testing.assert_allclose(x, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("smoother", ["tri_x", "tri_y", "adi"])
@pytest.mark.parametrize("kl", [(1, 1), (3, 6), (7, 2), (7, 7)])
def test_tri_damping_factor_closed_form(smoother, kl):
    """Sine modes are eigenvectors of A and of both line parts (Kronecker
    sums), so one step with b = 0 scales mode (k, l) by 1 - omega lam_A / lam_T
    (TRIx: lam_T = 4 ex/hx^2 sin^2(k pi hx/2) + 2 ey/hy^2; TRIy symmetric; ADI
    the product of the two)."""
    g = O.Grid(9, 9)
    ex, ey, omega = 0.05, 1.3, 0.7
    k, l = kl
    sx = 4 * ex / g.hx**2 * math.sin(k * math.pi * g.hx / 2) ** 2
    sy = 4 * ey / g.hy**2 * math.sin(l * math.pi * g.hy / 2) ** 2
    fx = 1 - omega * (sx + sy) / (sx + 2 * ey / g.hy**2)
    fy = 1 - omega * (sx + sy) / (sy + 2 * ex / g.hx**2)
    factor = {"tri_x": fx, "tri_y": fy, "adi": fx * fy}[smoother]
    h = O.hierarchy_5pt(g, ex, ey, O.Options(smoother=smoother, omega=omega), levels=2)
    s = sine_mode(g, k, l)
    out = O.smooth(h, 0, s, np.zeros_like(s), 1)
    np.testing.assert_allclose(out, factor * s, rtol=0, atol=1e-12 * np.abs(s).max())


def zebra_block_lower(g, A, direction):
    """Dense preconditioner of one GSTRI step: A with the couplings from each
    node to nodes of a later line colour removed (lines of colour 0 first)."""
    Ad = A.toarray()
    Jg, Ig = np.meshgrid(np.array(g.uy), np.array(g.ux), indexing="ij")  # stored j and i of each unknown
    key = (Jg if direction == "x" else Ig).reshape(-1) % 2
    M = Ad.copy()
    for p in range(len(key)):
        for q in range(len(key)):
            if key[q] > key[p]:
                M[p, q] = 0.0
    return M


@pytest.mark.parametrize("direction", ["x", "y"])
@pytest.mark.parametrize("case", ["5pt", "q1"])
def test_gstri_step_is_block_gauss_seidel(direction, case):
    """One GSTRI step equals x + M^{-1} (b - A x) with M the block lower
    triangular part of A in zebra line order (dense solve)."""
    rng = np.random.default_rng(5)
    g = O.Grid(9, 9)
    if case == "5pt":
        A = O.laplace5(g, 0.2, 1.0)
    else:
        kx = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        A = O.assemble_q1(g, kx, kx)
    x = rng.standard_normal(g.n_unknowns)
    b = rng.standard_normal(g.n_unknowns)
    got = O.line_gs_step(A, x, b, O.line_colour_sets(g, direction))
    M = zebra_block_lower(g, A, direction)
    want = x + np.linalg.solve(M, b - A @ x)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("direction", ["x", "y"])
def test_lines_of_one_colour_do_not_couple(direction):
    """A restricted to one zebra colour is block diagonal by lines (9-point)."""
    g = O.Grid(9, 9)
    kx = np.exp(np.random.default_rng(2).standard_normal((g.ncy, g.ncx)))
    A = O.assemble_q1(g, kx, kx)
    I, J = O._unknown_ij(g)
    line = J if direction == "x" else I
    for s in O.line_colour_sets(g, direction):
        sub = A[s][:, s].tocoo()
        assert np.all(line[s][sub.row] == line[s][sub.col])


@pytest.mark.parametrize("n", [17, 33, 65])
def test_line_smoother_cycle_is_robust_to_anisotropy(n):
    """The paper's point about line smoothers: with eps = 1e-3 (strong coupling
    along y) the F-cycle with y-line Gauss-Seidel reduces the residual by a
    large factor per cycle, independently of h, while point red-black
    Gauss-Seidel barely does (asymptotic rate from a random start, b = 0)."""
    g = O.Grid(n, n)
    x0 = g.pack(W.uniform_field(n, n, 7))
    rate = {}
    for sm in ("gstri_y", "gsadi", "rbgs"):
        h = O.hierarchy_5pt(g, 1e-3, 1.0, O.Options(smoother=sm))
        r = O.solve(h, np.zeros_like(x0), x0, 1e-300, 6)
        rate[sm] = (r.history[-1] / r.history[-3]) ** 0.5
    assert rate["gstri_y"] < 0.05 and rate["gsadi"] < 0.05
    assert rate["rbgs"] > 0.5


def test_line_smoother_rate_matches_cycle_matrix():
    """On 9^2 the asymptotic rate of GSTRIy cycles equals the spectral radius
    of the dense cycle matrix (the cycle is a fixed linear map)."""
    g = O.Grid(9, 9)
    h = O.hierarchy_5pt(g, 0.05, 1.0, O.Options(smoother="gstri_y"))
    rho = max(abs(np.linalg.eigvals(O.cycle_matrix(h, "F"))))
    x0 = g.pack(W.uniform_field(9, 9, 7))
    r = O.solve(h, np.zeros_like(x0), x0, 1e-300, 30)
    rate = (r.history[-1] / r.history[-11]) ** 0.1
    assert abs(rate - rho) <= 0.05 * rho


def test_tri_y_cycle_converges_on_anisotropic_problem():
    """A TRIy-smoothed F-cycle (omega 0.8) solves the eps = 1e-3 problem on
    65^2 to 1e-10 in a handful of cycles; TRIx (the wrong direction) does not."""
    g = O.Grid(65, 65)
    b = np.random.default_rng(0).standard_normal(g.n_unknowns)
    cyc = {}
    for sm in ("tri_y", "tri_x"):
        h = O.hierarchy_5pt(g, 1e-3, 1.0, O.Options(smoother=sm, omega=0.8))
        r = O.solve(h, b, np.zeros_like(b), 1e-10, 40)
        cyc[sm] = r.cycles if r.status == O.OK else None
    assert cyc["tri_y"] is not None and cyc["tri_y"] <= 12
    assert cyc["tri_x"] is None
