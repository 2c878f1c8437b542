"""Pins of the CPU oracle against closed forms, library routines, brute force
and invariants fixed by the paper and by the mathematics (no GPU).

Each test names the part of the oracle it pins and what it is pinned to.
"""

import math

import numpy as np
import pytest
import scipy.interpolate as si
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import mg_oracle as O
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def sine_mode(g, k, l):
    X, Y = W.node_coords(g.nx, g.ny, g.periodic_y, g.lx, g.ly)
    return g.pack(np.sin(k * np.pi * X / g.lx) * np.sin(l * np.pi * Y / g.ly))


# ----------------------------------------------------------------- 5-point operator


@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
@pytest.mark.parametrize("kl", [(1, 1), (3, 7), (15, 2), (15, 15)])
def test_laplace5_eigenpairs(eps, kl):
    """A s_kl = lambda_kl s_kl with lambda_kl = (4/h^2)(eps sin^2(k pi h/2) + sin^2(l pi h/2))."""
    g = O.Grid(17, 17)
    k, l = kl
    s = sine_mode(g, k, l)
    lam = 4.0 / g.hx**2 * (eps * math.sin(k * math.pi * g.hx / 2) ** 2 + math.sin(l * math.pi * g.hy / 2) ** 2)
    As = O.laplace5(g, eps, 1.0) @ s
    np.testing.assert_allclose(As, lam * s, rtol=0, atol=1e-12 * lam * np.abs(s).max())


def test_laplace5_rectangular_spacing():
    """Different hx, hy: eigenvalue (4/hx^2) eps sin^2 + (4/hy^2) sin^2."""
    g = O.Grid(9, 17, lx=2.0, ly=1.0)
    s = sine_mode(g, 3, 5)
    lam = 4 / g.hx**2 * 0.5 * math.sin(3 * math.pi * g.hx / 4) ** 2 + 4 / g.hy**2 * math.sin(5 * math.pi * g.hy / 2) ** 2
    np.testing.assert_allclose(O.laplace5(g, 0.5, 1.0) @ s, lam * s, atol=1e-12 * lam)


def test_laplace5_periodic_y_eigenpairs():
    """Periodic y: sin(k pi x) cos(2 pi m y) with eigenvalue (4/hx^2) sin^2(k pi hx/2) + (4/hy^2) sin^2(pi m hy)."""
    g = O.Grid(9, 16, periodic_y=True)
    X, Y = W.node_coords(g.nx, g.ny, True)
    for k, m in [(1, 0), (2, 3), (7, 8)]:
        s = g.pack(np.sin(k * np.pi * X) * np.cos(2 * np.pi * m * Y))
        lam = 4 / g.hx**2 * math.sin(k * math.pi * g.hx / 2) ** 2 + 4 / g.hy**2 * math.sin(math.pi * m * g.hy) ** 2
        np.testing.assert_allclose(O.laplace5(g) @ s, lam * s, atol=1e-11 * lam)


# ----------------------------------------------------------------- Q1 operator


def test_q1_isotropic_constant_stencil():
    """Constant a = 1: interior row is (1/(3h^2)) [-1 -1 -1; -1 8 -1; -1 -1 -1]."""
    g = O.Grid(9, 9)
    A = O.assemble_q1(g, np.ones((8, 8)), np.ones((8, 8))).toarray()
    idx = O._unknown_index(g)
    row = A[idx[4, 4]]
    h2 = g.hx**2
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            want = 8.0 / (3 * h2) if (di, dj) == (0, 0) else -1.0 / (3 * h2)
            assert abs(row[idx[4 + dj, 4 + di]] - want) < 1e-12 * 8 / (3 * h2)
    assert abs(row.sum()) < 1e-9


def test_q1_constant_tensor_form():
    """Constant kx, ky: A = kx T (x) M + ky M (x) T with T = (-1, 2, -1)/h^2, M = (1/6, 2/3, 1/6)."""
    g = O.Grid(9, 13, lx=1.0, ly=1.5)
    kx, ky = 2.5, 0.3
    A = O.assemble_q1(g, np.full((12, 8), kx), np.full((12, 8), ky)).toarray()
    def tm(n, h):
        m = n - 2
        T = (np.diag(2 * np.ones(m)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) / h**2
        M = np.diag(2 / 3 * np.ones(m)) + np.diag(np.ones(m - 1) / 6, 1) + np.diag(np.ones(m - 1) / 6, -1)
        return T, M
    Tx, Mx = tm(g.nx, g.hx)
    Ty, My = tm(g.ny, g.hy)
    ref = kx * np.kron(My, Tx) + ky * np.kron(Ty, Mx)
    np.testing.assert_allclose(A, ref, atol=1e-10 * np.abs(ref).max())


def test_q1_brute_force_dense_assembly():
    """Variable coefficients: every entry equals the bilinear form
    sum_cells int (kx phi_p,x phi_q,x + ky phi_p,y phi_q,y) / (hx hy), integrated
    with 3x3 Gauss quadrature from the bilinear hat functions (not from K1, M1)."""
    g = O.Grid(5, 6, periodic_y=False, lx=1.0, ly=2.0)
    rng = np.random.default_rng(0)
    kx = rng.uniform(0.5, 2, (g.ncy, g.ncx))
    ky = rng.uniform(0.5, 2, (g.ncy, g.ncx))
    A = O.assemble_q1(g, kx, ky).toarray()
    gp, gw = np.polynomial.legendre.leggauss(3)
    gp = 0.5 * (gp + 1)
    gw = 0.5 * gw
    idx = O._unknown_index(g)
    ref = np.zeros_like(A)
    for cj in range(g.ncy):
        for ci in range(g.ncx):
            for jp in (cj, cj + 1):
                for ip in (ci, ci + 1):
                    for jq in (cj, cj + 1):
                        for iq in (ci, ci + 1):
                            if idx[jp, ip] < 0 or idx[jq, iq] < 0:
                                continue
                            val = 0.0
                            for s, ws in zip(gp, gw):
                                for t, wt in zip(gp, gw):
                                    def hat(i, j):  # value and gradient at local (s, t)
                                        fx = s if i == ci + 1 else 1 - s
                                        fy = t if j == cj + 1 else 1 - t
                                        dx = (1 if i == ci + 1 else -1) / g.hx
                                        dy = (1 if j == cj + 1 else -1) / g.hy
                                        return dx * fy, fx * dy
                                    px, py = hat(ip, jp)
                                    qx, qy = hat(iq, jq)
                                    val += ws * wt * (kx[cj, ci] * px * qx + ky[cj, ci] * py * qy)
                            ref[idx[jp, ip], idx[jq, iq]] += val  # area hx*hy cancels the FD scaling
    np.testing.assert_allclose(A, ref, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())


def test_q1_row_equals_assembled_rows():
    """Single-row assembly (used to sample very large grids) equals rows of the assembled matrix."""
    for g in (O.Grid(9, 8, periodic_y=True), O.Grid(9, 9)):
        rng = np.random.default_rng(12)
        kx = rng.uniform(0.5, 2, (g.ncy, g.ncx))
        ky = rng.uniform(0.5, 2, (g.ncy, g.ncx))
        A = O.assemble_q1(g, kx, ky).toarray()
        idx = O._unknown_index(g)
        for j in g.uy:
            for i in g.ux:
                row = O.q1_row(g, kx, ky, i, j)
                dense = np.zeros(g.n_unknowns)
                for (jq, iq), v in row.items():
                    dense[idx[jq, iq]] += v
                np.testing.assert_allclose(dense, A[idx[j, i]], atol=1e-12 * np.abs(A).max())


def test_q1_separable_equals_elementwise():
    g = O.Grid(9, 8, periodic_y=True)
    kx, ky = W.annulus_cell_coefficients(9)
    A1 = O.assemble_q1(g, np.tile(kx, (g.ncy, 1)), np.tile(ky, (g.ncy, 1)))
    A2 = O.assemble_q1_separable(g, kx, ky)
    np.testing.assert_allclose(A1.toarray(), A2.toarray(), atol=1e-12 * abs(A1).max())


def test_q1_periodic_row_sums_zero():
    """With no Dirichlet boundary involved (full periodic rows away from x-boundary), rows sum to 0."""
    g = O.Grid(9, 8, periodic_y=True)
    rng = np.random.default_rng(1)
    A = O.assemble_q1(g, rng.uniform(1, 2, (8, 8)), rng.uniform(1, 2, (8, 8))).toarray()
    idx = O._unknown_index(g)
    for j in range(8):
        for i in range(2, 7):
            assert abs(A[idx[j, i]].sum()) < 1e-10 * abs(A[idx[j, i], idx[j, i]])


@pytest.mark.slow
def test_annulus_manufactured_second_order():
    """Mapped annulus: nodal max error of the direct solution falls as h^2
    (rate 2 +- 0.1 over three refinements), pinning the coefficients r, 1/r of
    the mapping, the Jacobian in the right-hand side and the Q1 assembly."""
    errs = []
    for n in (33, 65, 129):
        g = O.Grid(n, n - 1, periodic_y=True)
        kx, ky = W.annulus_cell_coefficients(n)
        A = O.assemble_q1_separable(g, kx, ky)
        b, u = W.annulus_manufactured(n, n - 1)
        x = spla.spsolve(A.tocsc(), g.pack(b))
        errs.append(np.abs(x - g.pack(u)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - 2) < 0.1 for r in rates), (errs, rates)


# ----------------------------------------------------------------- transfers


@pytest.mark.parametrize("kl", [(1, 1), (3, 5), (7, 2)])
def test_full_weighting_symbol(kl):
    """R s_kl = cos^2(k pi h/2) cos^2(l pi h/2) s_kl on the coarse grid, exactly."""
    g = O.Grid(17, 17)
    gc = g.coarse()
    k, l = kl
    Rs = O.restriction(g) @ sine_mode(g, k, l)
    fac = math.cos(k * math.pi * g.hx / 2) ** 2 * math.cos(l * math.pi * g.hy / 2) ** 2
    np.testing.assert_allclose(Rs, fac * sine_mode(gc, k, l), atol=1e-14)


@pytest.mark.parametrize("periodic", [False, True])
def test_prolongation_is_bilinear_interpolation(periodic):
    """P e equals the piecewise-bilinear interpolant of the coarse nodal values,
    evaluated at the fine nodes by scipy's RegularGridInterpolator."""
    g = O.Grid(17, 16, periodic_y=True) if periodic else O.Grid(17, 9)
    gc = g.coarse()
    rng = np.random.default_rng(3)
    ec = rng.standard_normal(gc.n_unknowns)
    E = gc.unpack(ec)
    xc = np.arange(gc.nx) * gc.hx
    yc = np.arange(gc.ny) * gc.hy
    if periodic:
        E = np.vstack([E, E[:1]])
        yc = np.append(yc, gc.ny * gc.hy)
    interp = si.RegularGridInterpolator((yc, xc), E, method="linear")
    X, Y = W.node_coords(g.nx, g.ny, g.periodic_y)
    ref = interp(np.stack([Y.ravel(), X.ravel()], axis=1)).reshape(g.ny, g.nx)
    np.testing.assert_allclose(O.prolongation(g) @ ec, g.pack(ref), atol=1e-14)


def test_restriction_is_quarter_transpose():
    g = O.Grid(17, 16, periodic_y=True)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(g.n_unknowns)
    v = rng.standard_normal(g.coarse().n_unknowns)
    R, P = O.restriction(g), O.prolongation(g)
    assert abs((R @ u) @ v - 0.25 * u @ (P @ v)) < 1e-12 * np.linalg.norm(u) * np.linalg.norm(v)


# ----------------------------------------------------------------- Galerkin coarse operators


def test_galerkin_of_5pt_laplacian_closed_form():
    """R A_h P for the 5-point Laplacian: (1/H^2)[-1/4 -1/2 -1/4; -1/2 3 -1/2; -1/4 -1/2 -1/4]."""
    g = O.Grid(17, 17)
    Ac = (O.restriction(g) @ O.laplace5(g) @ O.prolongation(g)).toarray()
    gc = g.coarse()
    idx = O._unknown_index(gc)
    H2 = gc.hx**2
    st = np.array([[-0.25, -0.5, -0.25], [-0.5, 3.0, -0.5], [-0.25, -0.5, -0.25]]) / H2
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            assert abs(Ac[idx[4, 4], idx[4 + dj, 4 + di]] - st[dj + 1, di + 1]) < 1e-10 * 3 / H2


@pytest.mark.parametrize("periodic", [False, True])
def test_galerkin_q1_constant_equals_rediscretised(periodic):
    """Constant-coefficient Q1: R A_h P equals the Q1 matrix rediscretised at H, exactly."""
    g = O.Grid(17, 16, periodic_y=True) if periodic else O.Grid(17, 17)
    kx, ky = 1.7, 0.4
    Ah = O.assemble_q1(g, np.full((g.ncy, g.ncx), kx), np.full((g.ncy, g.ncx), ky))
    gc = g.coarse()
    AH = O.assemble_q1(gc, np.full((gc.ncy, gc.ncx), kx), np.full((gc.ncy, gc.ncx), ky))
    Ag = O.restriction(g) @ Ah @ O.prolongation(g)
    np.testing.assert_allclose(Ag.toarray(), AH.toarray(), atol=1e-10 * abs(AH).max())


def test_galerkin_variable_symmetric_9pt():
    g = O.Grid(17, 17)
    rng = np.random.default_rng(5)
    a = np.exp(rng.standard_normal((16, 16)))
    h = O.hierarchy_q1(g, a, a)
    for A in h.A:
        D = A.toarray()
        np.testing.assert_allclose(D, D.T, atol=1e-12 * np.abs(D).max())
    # coarse operators keep a 9-point pattern
    Ac = h.A[1].toarray()
    gc = h.grids[1]
    idx = O._unknown_index(gc)
    nz = np.nonzero(Ac[idx[3, 3]])[0]
    assert len(nz) == 9


# ----------------------------------------------------------------- smoothers


def test_jacobi_mode_damping_closed_form():
    """One damped-Jacobi sweep with b = 0 scales s_kl by 1 - 2 omega (eps s_k + s_l)/(1 + eps),
    s_k = sin^2(k pi h/2); the high-frequency maximum at omega = 0.8, eps = 1 is 0.6 (LFA)."""
    g = O.Grid(17, 17)
    eps, om = 0.3, 0.8
    A = O.laplace5(g, eps, 1.0)
    d = A.diagonal()
    for k, l in [(1, 1), (5, 9), (16, 3)]:
        s = sine_mode(g, k, l)
        sk = math.sin(k * math.pi * g.hx / 2) ** 2
        sl = math.sin(l * math.pi * g.hy / 2) ** 2
        fac = 1 - 2 * om * (eps * sk + sl) / (1 + eps)
        np.testing.assert_allclose(O.jacobi_step(A, d, s, 0 * s, om), fac * s, atol=1e-13)
    # high-frequency maximum on a 64^2 grid (k or l >= 32): attained at |1 - 0.8 * 2| = 0.6 in the limit
    n = 64
    best = 0.0
    for k in range(1, n):
        for l in range(1, n):
            if max(k, l) >= n // 2:
                sk = math.sin(k * math.pi / (2 * n)) ** 2
                sl = math.sin(l * math.pi / (2 * n)) ** 2
                best = max(best, abs(1 - 0.8 * (sk + sl)))
    assert abs(best - 0.6) < 1e-3


@pytest.mark.parametrize("ncol,periodic", [(2, False), (4, False), (2, True), (4, True)])
def test_coloured_gs_equals_permuted_triangular_solve(ncol, periodic):
    """A coloured GS step equals x + (D + L)^{-1} (b - A x) with L the strictly
    lower triangle of A in colour-permuted order (dense, brute force)."""
    g = O.Grid(9, 8, periodic_y=True) if periodic else O.Grid(9, 9)
    rng = np.random.default_rng(6)
    if ncol == 2:
        A = O.laplace5(g, 0.3, 1.0)
    else:
        a = np.exp(rng.standard_normal((g.ncy, g.ncx)))
        A = O.assemble_q1(g, a, a)
    cols = O.colour_sets(g, ncol)
    perm = np.concatenate(cols)
    Ad = A.toarray()[np.ix_(perm, perm)]
    x = rng.standard_normal(g.n_unknowns)
    b = rng.standard_normal(g.n_unknowns)
    DL = np.tril(Ad)
    xp = x[perm] + sla.solve_triangular(DL, b[perm] - Ad @ x[perm], lower=True)
    ref = np.empty_like(x)
    ref[perm] = xp
    got = O.coloured_gs_step(A, A.diagonal(), x, b, cols)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_colours_do_not_couple():
    """No two nodes of one colour are coupled (so a colour's update is order-free)."""
    g = O.Grid(9, 8, periodic_y=True)
    a = np.ones((g.ncy, g.ncx))
    A = O.assemble_q1(g, a, a).tocsr()
    for c in O.colour_sets(g, 4):
        sub = A[c][:, c].toarray()
        assert np.count_nonzero(sub - np.diag(np.diag(sub))) == 0
    A5 = O.laplace5(g).tocsr()
    for c in O.colour_sets(g, 2):
        sub = A5[c][:, c].toarray()
        assert np.count_nonzero(sub - np.diag(np.diag(sub))) == 0


def test_jacobi_omega_too_large_diverges():
    """||I - omega D^{-1} A|| > 1 for omega = 2.5 (the convergence condition of the Smoothers section)."""
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="jacobi", omega=2.5))
    b = np.random.default_rng(0).standard_normal(g.n_unknowns)
    r = O.solve(h, b, np.zeros_like(b), 1e-10, 50)
    assert r.status == O.DIVERGED


def test_single_level_rate_degrades_as_h_squared():
    """Smoothing alone converges as 1 - O(h^2) for Jacobi and GS: halving h quarters 1 - rho."""
    rates = []
    for n in (17, 33):
        g = O.Grid(n, n)
        A = O.laplace5(g)
        d = A.diagonal()
        cols = O.colour_sets(g, 2)
        x = sine_mode(g, 1, 1)  # the slowest mode
        y = O.coloured_gs_step(A, d, x, 0 * x, cols)
        y2 = O.coloured_gs_step(A, d, y, 0 * x, cols)
        rates.append(np.linalg.norm(y2) / np.linalg.norm(y))
    ratio = (1 - rates[0]) / (1 - rates[1])
    assert 3.5 < ratio < 4.5, (rates, ratio)


# ----------------------------------------------------------------- coarse solve


def test_coarse_solve_single_unknown():
    g = O.Grid(3, 3)
    h = O.hierarchy_5pt(g)
    assert h.nlevels == 1
    gvec = np.array([1.7])
    np.testing.assert_allclose(O.coarse_solve(h, gvec), gvec / h.A[0].diagonal(), rtol=1e-15)


def test_coarse_solve_periodic_twelve_unknowns():
    g = O.Grid(5, 4, periodic_y=True)
    kx, ky = W.annulus_cell_coefficients(5)
    h = O.hierarchy_q1(g, kx, ky, separable=True)
    assert h.grids[-1].n_unknowns == 12
    rhs = np.random.default_rng(7).standard_normal(12)
    x = O.coarse_solve(h, rhs)
    assert np.linalg.norm(h.A[0] @ x - rhs) <= 1e-14 * np.linalg.norm(rhs) * 10


# ----------------------------------------------------------------- cycle


def _dense_error_propagators(h, kind):
    """Error propagation of the recursive algorithm written as dense matrices:
    E_V(l) = S_post (I - P (I - E_V(l+1)) A_{l+1}^{-1} R A_l) S_pre,
    E_F(l) = S_post (I - P (I - E_V(l+1) E_F(l+1)) A_{l+1}^{-1} R A_l) S_pre,
    E_W(l) = S_post (I - P (I - E_W(l+1)^2) A_{l+1}^{-1} R A_l) S_pre,
    E(coarsest) = 0; S from the smoother's C (I - omega D^{-1} A, or I - (D + L)^{-1} A per colour order)."""
    L = h.nlevels
    def S(l):
        A = h.A[l].toarray()
        n = A.shape[0]
        if h.opts.smoother == "jacobi":
            return np.eye(n) - h.opts.omega * A / np.diag(A)[:, None]
        perm = np.concatenate(h.colours[l])
        Q = np.eye(n)[perm]
        Ap = Q @ A @ Q.T
        Sp = np.eye(n) - sla.solve_triangular(np.tril(Ap), Ap, lower=True)
        return Q.T @ Sp @ Q
    EV = [None] * L
    EF = [None] * L
    EW = [None] * L
    EV[L - 1] = np.zeros((h.grids[-1].n_unknowns,) * 2)
    EF[L - 1] = EV[L - 1]
    EW[L - 1] = EV[L - 1]
    for l in range(L - 2, -1, -1):
        A = h.A[l].toarray()
        Ac = h.A[l + 1].toarray()
        R, P = h.R[l].toarray(), h.P[l].toarray()
        Sl = S(l)
        Spre = np.linalg.matrix_power(Sl, h.opts.nu_pre)
        Spost = np.linalg.matrix_power(Sl, h.opts.nu_post)
        cgc = np.linalg.solve(Ac, R @ A)
        I = np.eye(A.shape[0])
        EV[l] = Spost @ (I - P @ (np.eye(Ac.shape[0]) - EV[l + 1]) @ cgc) @ Spre
        EF[l] = Spost @ (I - P @ (np.eye(Ac.shape[0]) - EV[l + 1] @ EF[l + 1]) @ cgc) @ Spre
        EW[l] = Spost @ (I - P @ (np.eye(Ac.shape[0]) - EW[l + 1] @ EW[l + 1]) @ cgc) @ Spre
    return {"F": EF, "V": EV, "W": EW}[kind][0]


@pytest.mark.parametrize("smoother,levels", [("rbgs", 3), ("jacobi", 4), ("rbgs", 2)])
def test_cycle_matrix_equals_dense_recursion(smoother, levels):
    """The oracle's F-, V- and W-cycle iteration matrices equal the dense
    error-propagation recursion; with 2 levels F = V = W = two-grid."""
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, 0.5, 1.0, O.Options(smoother=smoother, nu_pre=2, nu_post=1), levels=levels)
    for kind in ("F", "V", "W"):
        M = O.cycle_matrix(h, kind)
        E = _dense_error_propagators(h, kind)
        np.testing.assert_allclose(M, E, atol=1e-11)
    if levels == 2:
        np.testing.assert_allclose(O.cycle_matrix(h, "F"), O.cycle_matrix(h, "V"), atol=1e-14)
        np.testing.assert_allclose(O.cycle_matrix(h, "W"), O.cycle_matrix(h, "V"), atol=1e-14)


def test_w_cycle_rate_between_two_grid_and_v():
    """W-cycles come closer to the two-grid rate than V-cycles: on 33^2
    Poisson with red-black GS 1/1, rho(two-grid) <= rho(W) <= rho(V)."""
    g = O.Grid(33, 33)
    opts = O.Options(smoother="rbgs", nu_pre=1, nu_post=1)
    rho = {}
    for kind, levels in (("two-grid", 2), ("W", 0), ("V", 0)):
        h = O.hierarchy_5pt(g, 1.0, 1.0, opts, levels=levels)
        rho[kind] = max(abs(np.linalg.eigvals(O.cycle_matrix(h, "V" if kind == "two-grid" else kind))))
    assert rho["two-grid"] <= rho["W"] + 1e-12 <= rho["V"] + 2e-12


def test_cycle_matrix_q1_gs4c_dense_recursion():
    g = O.Grid(9, 8, periodic_y=True)
    kx, ky = W.annulus_cell_coefficients(9)
    h = O.hierarchy_q1(g, np.tile(kx, (8, 1)), np.tile(ky, (8, 1)), O.Options(smoother="gs4c"))
    np.testing.assert_allclose(O.cycle_matrix(h, "F"), _dense_error_propagators(h, "F"), atol=1e-11)


def test_f_cycle_spectral_radius_below_one():
    for n in (17, 33):
        g = O.Grid(n, n)
        h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="jacobi", omega=0.8))
        rho = max(abs(np.linalg.eigvals(O.cycle_matrix(h, "F"))))
        assert rho < 0.2, rho


def test_cycle_affine():
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, 0.1, 1.0, O.Options(smoother="rbgs"))
    rng = np.random.default_rng(8)
    x, y = rng.standard_normal((2, g.n_unknowns))
    z = np.zeros(g.n_unknowns)
    lhs = O.mg_cycle(h, 0, 2.0 * x - 3.0 * y, z)
    rhs = 2.0 * O.mg_cycle(h, 0, x, z) - 3.0 * O.mg_cycle(h, 0, y, z)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


# ----------------------------------------------------------------- whole solve


@pytest.mark.parametrize("eps", [1.0, 0.1])
def test_manufactured_solution_closed_form_error(eps):
    """u = sin(pi x) sin(pi y): the discrete solution is [(x/sin x)]^2 u with x = pi h/2,
    so the converged max error is (x/sin x)^2 - 1 = 2.00822e-4 at h = 1/64, for any eps."""
    n = 65
    g = O.Grid(n, n)
    f, u = W.manufactured_sine(n, eps)
    h = O.hierarchy_5pt(g, eps, 1.0, O.Options(smoother="jacobi", omega=0.8))
    r = O.solve(h, g.pack(f), np.zeros(g.n_unknowns), 1e-12, 200)
    assert r.status == O.OK
    xh = math.pi / 128
    want = (xh / math.sin(xh)) ** 2 - 1
    assert abs(want - 2.00822e-4) < 1e-9
    err = np.abs(r.x - g.pack(u)).max()
    assert abs(err - want) < 1e-10, (err, want)


def test_poisson65_matches_dense_solve():
    """65^2 Jacobi F-cycle to 1e-10 equals numpy.linalg.solve on the dense Kronecker-sum matrix within kappa * tol."""
    n = 65
    g = O.Grid(n, n)
    b = g.pack(W.normal_field(n, n, 0))
    m = n - 2
    T = (np.diag(2 * np.ones(m)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) * (n - 1) ** 2
    Ad = np.kron(np.eye(m), T) + np.kron(T, np.eye(m))
    xd = np.linalg.solve(Ad, b)
    h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="jacobi", omega=0.8))
    r = O.solve(h, b, np.zeros_like(b), 1e-10, 100)
    assert r.status == O.OK and r.cycles < 20
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(r.x - xd) <= kappa * 1e-10 * np.linalg.norm(xd)
    assert np.abs(r.x - xd).max() < 1e-12 * 1e3 * np.abs(xd).max()


def test_not_converged_and_zero_rhs():
    g = O.Grid(33, 33)
    h = O.hierarchy_5pt(g, 1e-3, 1.0, O.Options(smoother="rbgs"))
    b = np.random.default_rng(1).standard_normal(g.n_unknowns)
    r = O.solve(h, b, np.zeros_like(b), 1e-10, 1)
    assert r.status == O.NOT_CONVERGED and r.cycles == 1
    r = O.solve(h, 0 * b, np.zeros_like(b), 1e-10, 5)
    assert r.status == O.OK and r.cycles == 0


def test_resume_equals_continuous():
    """The F-cycle is a stationary iteration: k cycles then m more equals k + m cycles."""
    g = O.Grid(33, 33)
    h = O.hierarchy_5pt(g, 0.01, 1.0, O.Options(smoother="rbgs"))
    b = np.random.default_rng(2).standard_normal(g.n_unknowns)
    a = O.solve(h, b, np.zeros_like(b), 1e-30, 5)
    c = O.solve(h, b, O.solve(h, b, np.zeros_like(b), 1e-30, 2).x, 1e-30, 3)
    np.testing.assert_array_equal(a.x, c.x)


def test_mixed_precision_converges_like_fp64():
    g = O.Grid(129, 129)
    b = g.pack(W.aniso_rhs(129, 2))
    for eps in (1.0, 0.1):
        h = O.hierarchy_5pt(g, eps, 1.0, O.Options(smoother="rbgs"))
        r64 = O.solve(h, b, np.zeros_like(b), 1e-10, 500)
        r32 = O.solve_mixed(h, b, np.zeros_like(b), 1e-10, 500)
        assert r32.status == O.OK
        assert r32.cycles <= r64.cycles + 2
        assert O.residual_norm(h, b, r32.x) <= 1e-10 * r32.history[0]


@pytest.mark.parametrize("inner", [1, 2, 3])
def test_mixed_inner_cycles_in_fp64_equal_plain_cycles(inner):
    """Defect correction with an FP64 inner hierarchy: one outer step with k
    inner cycles from e = 0 equals k plain cycles from x (the cycle is affine:
    cycle(x, b) = x + cycle(0, b - A x)), so the mixed form's inner loop is
    pinned against the plain cycle independently of FP32 rounding."""
    g = O.Grid(33, 33)
    h = O.hierarchy_5pt(g, 0.1, 1.0, O.Options(smoother="rbgs"))
    rng = np.random.default_rng(11)
    b, x0 = rng.standard_normal((2, g.n_unknowns))
    one = O.solve_mixed(h, b, x0, 1e-300, 1, h32=h, inner=inner)
    x = x0.copy()
    for _ in range(inner):
        x = O.mg_cycle(h, 0, x, b, "F")
    np.testing.assert_allclose(one.x, x, rtol=0, atol=1e-12 * np.abs(x).max())


def _energy_error(A, xs, v):
    e = v - xs
    return float(e @ (A @ e))


@pytest.mark.parametrize("eps", [1.0, 0.05])
def test_energy_weight_minimises_the_energy_error(eps):
    """The adaptive coarse-correction weight minimises ||x + w P v - x*||_A
    over w: E(w) is an exact quadratic, fitted through three points with x*
    from a dense solve, and its vertex equals energy_weight (a wrong sign, a
    plain (P v, P v) denominator or the residual in place of the defect moves
    it); no other w on a fine scan does better."""
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, eps, 1.0, O.Options(smoother="rbgs", nu_pre=1))
    A = h.A[0]
    rng = np.random.default_rng(12)
    b = rng.standard_normal(g.n_unknowns)
    xs = np.linalg.solve(A.toarray(), b)
    x = O.smooth(h, 0, rng.standard_normal(g.n_unknowns), b, 1)
    pe = O.coarse_correction(h, 0, x, b, "F")
    w = O.energy_weight(h, 0, x, b, pe)
    ws = np.array([-1.0, 0.5, 2.0])
    c2, c1, _ = np.polyfit(ws, [_energy_error(A, xs, x + t * pe) for t in ws], 2)
    assert abs(w - (-c1 / (2 * c2))) <= 1e-10 * abs(w)
    scan = np.linspace(w - 0.5, w + 0.5, 101)
    assert _energy_error(A, xs, x + w * pe) <= min(_energy_error(A, xs, x + t * pe) for t in scan) * (1 + 1e-12)


def test_energy_weight_of_exact_galerkin_two_grid_is_one():
    """With a Galerkin coarse operator A_c = R A P (P = 4 R^T) solved exactly,
    P A_c^-1 R d is the A-orthogonal projection of the error onto range(P), so
    the energy-minimising weight along it is exactly 1; with the rediscretised
    5-point coarse operator it is not."""
    g = O.Grid(17, 17)
    rng = np.random.default_rng(13)
    b, x = rng.standard_normal((2, g.n_unknowns))
    ws = {}
    for galerkin in (True, False):
        h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs"), levels=2, galerkin=galerkin)
        pe = O.coarse_correction(h, 0, x, b, "V")
        ws[galerkin] = O.energy_weight(h, 0, x, b, pe)
    assert abs(ws[True] - 1.0) <= 1e-12
    assert abs(ws[False] - 1.0) > 1e-3


def test_adaptive_cycle_lowers_the_energy_error_after_correction():
    """A cycle with the adaptive weight and no post-smoothing ends with an
    energy error no larger than the same cycle with omega_l = 1 (the weight
    minimises it along the same correction)."""
    g = O.Grid(33, 33)
    rng = np.random.default_rng(14)
    b, x0 = rng.standard_normal((2, g.n_unknowns))
    out = {}
    for adaptive in (False, True):
        h = O.hierarchy_5pt(g, 0.3, 1.0, O.Options(smoother="rbgs", nu_post=0, adaptive_omega=adaptive))
        out[adaptive] = O.mg_cycle(h, 0, x0, b, "F")
    xs = np.linalg.solve(h.A[0].toarray(), b)
    assert _energy_error(h.A[0], xs, out[True]) <= _energy_error(h.A[0], xs, out[False]) * (1 + 1e-12)


# ----------------------------------------------------------------- adjoint


def _grf_small(n, seed=5):
    return np.exp(W.gaussian_random_field(n - 1, seed))


def test_adjoint_gradient_matches_central_differences():
    """dL/da from the adjoint formula equals central FD of L(a) with direct solves (<= 1e-5 relative)."""
    n = 9
    g = O.Grid(n, n)
    a = _grf_small(n)
    f, us = W.manufactured_sine(n, 1.0)
    us = us * 1.3  # make u - u* sizeable
    u, lam, dLda, dLdf = O.adjoint_gradient(g, a, f, us)

    def loss(aa):
        A = O.assemble_q1(g, aa, aa)
        uu = spla.spsolve(A.tocsc(), g.pack(f))
        return 0.5 * np.sum((uu - g.pack(us)) ** 2)

    fd = np.zeros_like(a)
    for cj in range(g.ncy):
        for ci in range(g.ncx):
            tau = 1e-4 * np.abs(a).max()
            ap, am = a.copy(), a.copy()
            ap[cj, ci] += tau
            am[cj, ci] -= tau
            fd[cj, ci] = (loss(ap) - loss(am)) / (2 * tau)
    assert np.linalg.norm(dLda - fd) <= 1e-5 * np.linalg.norm(fd)


def test_adjoint_tangent_linear_dot_product():
    """<dL/da, da> equals the tangent-linear value (u - u*)^T (-A^{-1} (dA u)) from a forward-mode path."""
    n = 17
    g = O.Grid(n, n)
    a = _grf_small(n)
    f, us = W.manufactured_sine(n, 1.0)
    u, lam, dLda, _ = O.adjoint_gradient(g, a, f, 0.5 * us)
    da = np.random.default_rng(9).standard_normal(a.shape)
    A = O.assemble_q1(g, a, a)
    dA = O.assemble_q1(g, da, da)  # A is linear in a
    du = -spla.spsolve(A.tocsc(), dA @ g.pack(u))
    tl = (g.pack(u) - g.pack(0.5 * us)) @ du
    assert abs(np.sum(dLda * da) - tl) <= 1e-10 * abs(tl)


def test_adjoint_dL_df_is_lambda_dense():
    """dL/df = lam, checked by dense LU: dL/df = A^{-T} (u - u*) with b = f."""
    n = 17
    g = O.Grid(n, n)
    a = _grf_small(n)
    f, us = W.manufactured_sine(n, 1.0)
    u, lam, _, dLdf = O.adjoint_gradient(g, a, f, 0.7 * us)
    Ad = O.assemble_q1(g, a, a).toarray()
    ud = sla.lu_solve(sla.lu_factor(Ad), g.pack(f))
    ld = sla.lu_solve(sla.lu_factor(Ad.T), ud - g.pack(0.7 * us))
    np.testing.assert_allclose(g.pack(dLdf), ld, atol=1e-12 * np.abs(ld).max())


def test_vectorised_gradient_equals_loop():
    for g in (O.Grid(9, 9), O.Grid(9, 8, periodic_y=True)):
        rng = np.random.default_rng(10)
        u = W.zero_boundary(rng.standard_normal((g.ny, g.nx)), g.periodic_y)
        lam = W.zero_boundary(rng.standard_normal((g.ny, g.nx)), g.periodic_y)
        for part in ("a", "kx", "ky"):
            np.testing.assert_allclose(O.q1_coeff_grad_vectorised(g, u, lam, part),
                                       O.q1_coeff_grad(g, u, lam, part), atol=1e-10)


# ----------------------------------------------------------------- inputs


def test_grf_covariance():
    """The circulant-embedding field has unit variance and correlation exp(-d^2/(2 l^2))."""
    n = 128
    samples = np.stack([W.gaussian_random_field(n, s) for s in range(40)])
    var = samples.var()
    assert abs(var - 1.0) < 0.1
    lag = 13  # d = 13/128 ~ 0.1 = length
    c = np.mean(samples[:, :, :-lag] * samples[:, :, lag:])
    assert abs(c - math.exp(-((lag / n) ** 2) / (2 * 0.01))) < 0.08


def test_hierarchy_shapes():
    assert [(x.nx, x.ny) for x in O.hierarchy_grids(O.Grid(65, 65))] == [(65, 65), (33, 33), (17, 17), (9, 9), (5, 5), (3, 3)]
    gs = O.hierarchy_grids(O.Grid(4097, 4096, periodic_y=True))
    assert len(gs) == 11 and (gs[-1].nx, gs[-1].ny) == (5, 4)
    assert gs[0].n_unknowns == 4095 * 4096
    with pytest.raises(ValueError):
        O.hierarchy_grids(O.Grid(65, 65), levels=7)


# ----------------------------------------------------------------- nested-iteration start vector


def test_nested_start_two_levels_is_coarse_grid_solution():
    """With two levels the start is P A_1^{-1} R b (dense solve)."""
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, 0.3, 1.0, O.Options(), levels=2)
    b = np.random.default_rng(4).standard_normal(g.n_unknowns)
    want = h.P[0].toarray() @ np.linalg.solve(h.A[1].toarray(), h.R[0].toarray() @ b)
    np.testing.assert_allclose(O.nested_start(h, b), want, rtol=1e-12, atol=1e-13 * np.abs(want).max())


def test_nested_start_three_levels_composition():
    """With three levels: x_2 = A_2^{-1} R R b (dense), one cycle on level 1
    from P x_2 (its error propagation from the dense recursion), then P."""
    g = O.Grid(17, 17)
    h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="jacobi", omega=0.8, nu_pre=1, nu_post=1), levels=3)
    b = np.random.default_rng(5).standard_normal(g.n_unknowns)
    R0, R1, P0, P1 = (m.toarray() for m in (h.R[0], h.R[1], h.P[0], h.P[1]))
    A1, A2 = h.A[1].toarray(), h.A[2].toarray()
    b1 = R0 @ b
    x1_exact = np.linalg.solve(A1, b1)
    start1 = P1 @ np.linalg.solve(A2, R1 @ b1)
    # one two-grid cycle on level 1 (its coarse level is the exact coarsest solve):
    n1 = A1.shape[0]
    S = np.eye(n1) - 0.8 * A1 / np.diag(A1)[:, None]
    E = S @ (np.eye(n1) - P1 @ np.linalg.solve(A2, R1 @ A1)) @ S
    x1 = x1_exact + E @ (start1 - x1_exact)
    want = P0 @ x1
    np.testing.assert_allclose(O.nested_start(h, b), want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_nested_start_is_second_order_accurate():
    """Nested iteration reaches the discretisation's order: for the
    manufactured sine problem the start vector's distance to the discrete
    solution falls by 4 per halving of h (65^2, 129^2, 257^2), like the
    discretisation error itself, so cycles from it only need to remove a
    fixed factor of error on every grid."""
    errs = []
    for n in (65, 129, 257):
        g = O.Grid(n, n)
        h = O.hierarchy_5pt(g, 1.0, 1.0, O.Options(smoother="rbgs", cycle="F"))
        f, u = W.manufactured_sine(n)
        b = g.pack(f)
        x_disc = O.solve(h, b, np.zeros(g.n_unknowns), 1e-13, 50).x
        errs.append(np.abs(O.nested_start(h, b) - x_disc).max())
    for a, c in zip(errs, errs[1:]):
        assert 3.5 < a / c < 4.5, errs
