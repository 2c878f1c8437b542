"""Plain, slow, FP64 CPU oracle for the geometric-multigrid F-cycle.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this module imports nothing from the product path.

What it computes, and where the paper defines it (J. T. Wallis, "Methods toward
better Multigrid Solver Convergence", KAIST 2008):

* the discrete Poisson problem of the Abstract and the anisotropic operator
  -alpha u_xx - beta u_yy of the "Anisotropies" section, as the 5-point finite
  difference matrix, written out as a Kronecker sum;
* the coordinate-mapped (polar annulus -> unit square) operator of the
  Introduction's "Some Typical Problems" and of "Different coordinate systems",
  as a bilinear (Q1) finite-element matrix assembled element by element from
  per-cell coefficients;
* the preconditioned Richardson smoother x <- x - omega C^{-1}(A x - b) of the
  "Smoothers" section with C = D (Jacobi) and C = D + omega L (Gauss-Seidel at
  omega = 1, SOR otherwise, "The choice of C"; Options.sor), the Gauss-Seidel
  ordering being red-black (5-point) or four-colour (9-point) and L the
  couplings to earlier colours;
* the line smoothers of "The choice of C" and "Smoothing": TRI (C = the
  tridiagonal part of A along x or y lines, damped by omega), ADI (a TRI step
  along x then one along y), GSTRI (Gauss-Seidel over whole lines, each line
  solved exactly, lines in zebra order) and GSADI (GSTRI along x then y);
* the recursive algorithm MG(l, u, g) of "The Multigrid Technique" (pre-smooth,
  restrict the defect, solve recursively from a zero start, add the prolonged
  correction with omega_l = 1, post-smooth, exact solve on the coarsest level),
  run as the F-cycle the Abstract names;
* a start vector by nested iteration ("Start-Vector Choice");
* the stopping test on the relative residual, a mixed-precision
  defect-correction form, and the adjoint gradient of a least-squares loss with
  respect to the per-cell coefficient.

Every operator is an explicit ``scipy.sparse`` matrix built from its
definition (Kronecker products, element-by-element assembly, sparse triple
products) rather than a matrix-free stencil; library primitives used as steps
are sparse products, ``scipy.linalg.cho_factor``/``cho_solve`` and
``scipy.sparse.linalg.spsolve``.

Readings of passages the paper leaves open (all numbered as in the design
notes): F-cycle = standard F-cycle, coarse problem gets one F then one V cycle
from a zero start; omega_l = 1; full-weighting restriction and bilinear
prolongation P = 4 R^T; 5-point coarse operators rediscretised, 9-point coarse
operators Galerkin R A P; red = (i + j) even on stored level indices, red
before black; four colours (i mod 2, j mod 2) in the order (0,0), (1,0), (0,1),
(1,1); Dirichlet boundary nodes are not unknowns; a periodic direction has no
boundary nodes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Status values shared in meaning (not in code) with the library's C ABI.
OK, NOT_CONVERGED, DIVERGED = 0, 1, 2

DIVERGENCE_FACTOR = 1.0e6  # a cycle whose residual exceeds this times r0 is reported as divergence

# --------------------------------------------------------------------------- grid


@dataclass(frozen=True)
class Grid:
    """A tensor-product grid on [0, lx] x [0, ly] with stored nodes [ny][nx], x fastest.

    Dirichlet direction: n = 2^k m + 1 nodes, h = l / (n - 1), nodes 0 and n-1
    are boundary nodes (value 0, not unknowns).  Periodic direction (only y):
    n = 2^k m nodes, h = l / n, every node is an unknown and indices wrap.
    """

    nx: int
    ny: int
    periodic_y: bool = False
    lx: float = 1.0
    ly: float = 1.0

    @property
    def hx(self) -> float:
        return self.lx / (self.nx - 1)

    @property
    def hy(self) -> float:
        return self.ly / self.ny if self.periodic_y else self.ly / (self.ny - 1)

    @property
    def ux(self) -> range:
        """Stored x indices that are unknowns."""
        return range(1, self.nx - 1)

    @property
    def uy(self) -> range:
        return range(0, self.ny) if self.periodic_y else range(1, self.ny - 1)

    @property
    def n_unknowns(self) -> int:
        return len(self.ux) * len(self.uy)

    @property
    def ncx(self) -> int:
        """Number of cells along x."""
        return self.nx - 1

    @property
    def ncy(self) -> int:
        return self.ny if self.periodic_y else self.ny - 1

    def coarse(self) -> "Grid":
        ncx = (self.nx - 1) // 2 + 1
        ncy = self.ny // 2 if self.periodic_y else (self.ny - 1) // 2 + 1
        return Grid(ncx, ncy, self.periodic_y, self.lx, self.ly)

    def can_coarsen(self) -> bool:
        okx = (self.nx - 1) % 2 == 0 and self.nx >= 5
        if self.periodic_y:
            oky = self.ny % 2 == 0 and self.ny >= 8
        else:
            oky = (self.ny - 1) % 2 == 0 and self.ny >= 5
        return okx and oky

    # packing between stored arrays [ny][nx] and unknown vectors (row-major, x fastest)
    def pack(self, u: np.ndarray) -> np.ndarray:
        u = np.asarray(u).reshape(self.ny, self.nx)
        return np.ascontiguousarray(u[self.uy.start:self.uy.stop, 1:self.nx - 1]).reshape(-1)

    def unpack(self, v: np.ndarray, dtype=None) -> np.ndarray:
        v = np.asarray(v)
        out = np.zeros((self.ny, self.nx), dtype=dtype or v.dtype)
        out[self.uy.start:self.uy.stop, 1:self.nx - 1] = v.reshape(len(self.uy), len(self.ux))
        return out


def hierarchy_grids(g: Grid, levels: int = 0) -> list[Grid]:
    """Level shapes, finest first.  ``levels = 0`` coarsens as far as possible
    (3 nodes in a Dirichlet direction, 4 in a periodic one).  Grids of the
    multigrid algorithm: one per level l of MG(l, u, g)."""
    out = [g]
    while out[-1].can_coarsen() and (levels == 0 or len(out) < levels):
        out.append(out[-1].coarse())
    if levels and len(out) != levels:
        raise ValueError(f"grid {g.nx}x{g.ny} supports at most {len(out)} levels, asked for {levels}")
    return out


# --------------------------------------------------------------------------- 1-D building blocks


def _second_difference_1d(n_stored: int, h: float, periodic: bool) -> sp.csr_matrix:
    """(-1, 2, -1)/h^2 on the unknowns of one direction."""
    if periodic:
        n = n_stored
        rows, cols, vals = [], [], []
        for i in range(n):
            rows += [i, i, i]
            cols += [(i - 1) % n, i, (i + 1) % n]
            vals += [-1.0, 2.0, -1.0]
        return sp.csr_matrix((np.array(vals) / h**2, (rows, cols)), shape=(n, n))
    n = n_stored - 2
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr") / h**2


def _identity_1d(n_stored: int, periodic: bool) -> sp.csr_matrix:
    return sp.identity(n_stored if periodic else n_stored - 2, format="csr")


def _fw_1d(nf: int, periodic: bool) -> sp.csr_matrix:
    """1-D full weighting (1/4, 1/2, 1/4): coarse node I <- fine nodes 2I-1, 2I, 2I+1."""
    if periodic:
        nc = nf // 2
        rows, cols, vals = [], [], []
        for I in range(nc):
            for off, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
                rows.append(I)
                cols.append((2 * I + off) % nf)
                vals.append(w)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nc, nf))
    nc = (nf - 1) // 2 + 1
    rows, cols, vals = [], [], []
    for I in range(1, nc - 1):  # coarse unknowns; their fine support is interior
        for off, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            rows.append(I - 1)
            cols.append(2 * I + off - 1)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc - 2, nf - 2))


# --------------------------------------------------------------------------- operators


def laplace5(g: Grid, eps_x: float = 1.0, eps_y: float = 1.0) -> sp.csr_matrix:
    """5-point FD matrix of -(eps_x u_xx + eps_y u_yy) on the unknowns of ``g``:
    the Kronecker sum eps_x (I_y (x) T_x) + eps_y (T_y (x) I_x)  (Abstract's
    Poisson problem; anisotropic form of the "Anisotropies" section with
    alpha = eps_x, beta = eps_y)."""
    Tx = _second_difference_1d(g.nx, g.hx, False)
    Ty = _second_difference_1d(g.ny, g.hy, g.periodic_y)
    Ix = _identity_1d(g.nx, False)
    Iy = _identity_1d(g.ny, g.periodic_y)
    return (eps_x * sp.kron(Iy, Tx) + eps_y * sp.kron(Ty, Ix)).tocsr()


K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])  # 1-D unit stiffness
M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])  # 1-D unit mass


def q1_element_matrices(hx: float, hy: float) -> tuple[np.ndarray, np.ndarray]:
    """Element matrices of the x- and y-diffusion parts on one cell, divided by
    hx*hy ("FD scaling"), local node order (a, b) -> 2*b + a with a along x.
    Ex[(a,b),(a',b')] = K1[a,a'] M1[b,b'] / hx^2, Ey = M1[a,a'] K1[b,b'] / hy^2."""
    Ex = np.zeros((4, 4))
    Ey = np.zeros((4, 4))
    for a in range(2):
        for b in range(2):
            for a2 in range(2):
                for b2 in range(2):
                    Ex[2 * b + a, 2 * b2 + a2] = K1[a, a2] * M1[b, b2] / hx**2
                    Ey[2 * b + a, 2 * b2 + a2] = M1[a, a2] * K1[b, b2] / hy**2
    return Ex, Ey


def _unknown_index(g: Grid) -> np.ndarray:
    """Map stored node (j, i) -> unknown index, or -1 for a Dirichlet boundary node."""
    idx = -np.ones((g.ny, g.nx), dtype=np.int64)
    k = 0
    for j in g.uy:
        for i in g.ux:
            idx[j, i] = k
            k += 1
    return idx


def _cell_nodes(g: Grid, ci: int, cj: int) -> list[tuple[int, int]]:
    """Stored (j, i) of the 4 nodes of cell (cj, ci) in local order 2*b + a."""
    return [((cj + b) % g.ny if g.periodic_y else cj + b, ci + a) for b in range(2) for a in range(2)]


def assemble_q1(g: Grid, kx: np.ndarray, ky: np.ndarray) -> sp.csr_matrix:
    """Bilinear-FEM matrix of -div(diag(kx, ky) grad u), element by element
    from per-cell constants kx[cj][ci], ky[cj][ci] (shape [ncy][ncx]), divided by
    hx*hy, restricted to the unknowns.  This is the variable-coefficient
    operator that mapping a curved domain to the unit square produces."""
    kx = np.asarray(kx, dtype=np.float64).reshape(g.ncy, g.ncx)
    ky = np.asarray(ky, dtype=np.float64).reshape(g.ncy, g.ncx)
    Ex, Ey = q1_element_matrices(g.hx, g.hy)
    idx = _unknown_index(g)
    rows, cols, vals = [], [], []
    for cj in range(g.ncy):
        for ci in range(g.ncx):
            E = kx[cj, ci] * Ex + ky[cj, ci] * Ey
            nodes = _cell_nodes(g, ci, cj)
            for p, (jp, ip) in enumerate(nodes):
                rp = idx[jp, ip]
                if rp < 0:
                    continue
                for q, (jq, iq) in enumerate(nodes):
                    cq = idx[jq, iq]
                    if cq < 0:
                        continue
                    rows.append(rp)
                    cols.append(cq)
                    vals.append(E[p, q])
    n = g.n_unknowns
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def assemble_q1_separable(g: Grid, kx_of_x: np.ndarray, ky_of_x: np.ndarray) -> sp.csr_matrix:
    """Same matrix as :func:`assemble_q1` when the cell coefficients depend on
    the x cell index only (kx[cj][ci] = kx_of_x[ci]): the element sum factors
    into Kronecker products, A = M_y (x) K_x[kx] + K_y (x) M_x[ky], where K_x[k]
    and M_x[k] are the 1-D stiffness/hx^2 and mass matrices with cell weights k.
    Used for large annulus grids where element-by-element assembly is slow."""
    kx_of_x = np.asarray(kx_of_x, dtype=np.float64)
    ky_of_x = np.asarray(ky_of_x, dtype=np.float64)

    def weighted_1d(n_stored: int, weights: np.ndarray, local: np.ndarray, periodic: bool) -> sp.csr_matrix:
        ncell = n_stored if periodic else n_stored - 1
        rows, cols, vals = [], [], []
        for c in range(ncell):
            nodes = [c, (c + 1) % n_stored if periodic else c + 1]
            for a in range(2):
                for a2 in range(2):
                    rows.append(nodes[a])
                    cols.append(nodes[a2])
                    vals.append(weights[c] * local[a, a2])
        full = sp.csr_matrix((vals, (rows, cols)), shape=(n_stored, n_stored))
        if periodic:
            return full
        return full[1:n_stored - 1, 1:n_stored - 1]

    ones_y = np.ones(g.ncy)
    Kx = weighted_1d(g.nx, kx_of_x, K1, False) / g.hx**2
    Mx = weighted_1d(g.nx, ky_of_x, M1, False)
    My = weighted_1d(g.ny, ones_y, M1, g.periodic_y)
    Ky = weighted_1d(g.ny, ones_y, K1, g.periodic_y) / g.hy**2
    return (sp.kron(My, Kx) + sp.kron(Ky, Mx)).tocsr()


def assemble_q1_graded(g: Grid, xs, ys, kx: np.ndarray, ky: np.ndarray) -> sp.csr_matrix:
    """Bilinear-FEM matrix of -div(diag(kx, ky) grad u) on a tensor grid that
    is refined rather than equidistant (the anisotropically refined grids of
    the "Anisotropies" section; refinement toward one side in "Different
    coordinate systems"): node (i, j) at (xs[i], ys[j]), cell (ci, cj) of
    size hx_c = xs[ci+1] - xs[ci] by hy_c = ys[cj+1] - ys[cj] (Dirichlet y;
    xs, ys may be None for equidistant).  On that rectangle the x part of the
    element integral is kx hy_c/hx_c K1 (x) M1 and the y part ky hx_c/hy_c
    M1 (x) K1; the matrix is divided by hx0 hy0, the equidistant spacings
    (lx/(nx-1), and ly/(ny-1) or ly/ny for a periodic y), the scaling of
    :func:`assemble_q1`, which it equals on an equidistant grid."""
    assert not g.periodic_y or ys is None
    # cell boundaries: nx nodes along x; along y the ncy + 1 cell edges (a
    # periodic direction's last cell closes on node 0)
    xs = np.linspace(0.0, g.lx, g.nx) if xs is None else np.asarray(xs, dtype=np.float64)
    ys = np.linspace(0.0, g.ly, g.ncy + 1) if ys is None else np.asarray(ys, dtype=np.float64)
    kx = np.asarray(kx, dtype=np.float64).reshape(g.ncy, g.ncx)
    ky = np.asarray(ky, dtype=np.float64).reshape(g.ncy, g.ncx)
    hx0, hy0 = g.hx, g.hy
    Kx = np.zeros((4, 4))  # K1 (x) M1 and M1 (x) K1 in local order 2*b + a
    Ky = np.zeros((4, 4))
    for a in range(2):
        for b in range(2):
            for a2 in range(2):
                for b2 in range(2):
                    Kx[2 * b + a, 2 * b2 + a2] = K1[a, a2] * M1[b, b2]
                    Ky[2 * b + a, 2 * b2 + a2] = M1[a, a2] * K1[b, b2]
    idx = _unknown_index(g)
    rows, cols, vals = [], [], []
    for cj in range(g.ncy):
        hy = ys[cj + 1] - ys[cj]
        for ci in range(g.ncx):
            hx = xs[ci + 1] - xs[ci]
            E = (kx[cj, ci] * (hy / hx) * Kx + ky[cj, ci] * (hx / hy) * Ky) / (hx0 * hy0)
            nodes = _cell_nodes(g, ci, cj)
            for p_, (jp, ip) in enumerate(nodes):
                rp = idx[jp, ip]
                if rp < 0:
                    continue
                for q, (jq, iq) in enumerate(nodes):
                    cq = idx[jq, iq]
                    if cq < 0:
                        continue
                    rows.append(rp)
                    cols.append(cq)
                    vals.append(E[p_, q])
    n = g.n_unknowns
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def q1_row(g: Grid, kx: np.ndarray, ky: np.ndarray, i: int, j: int) -> dict:
    """Row of the Q1 matrix at unknown node (i, j): {(jq, iq): a_pq} over the
    unknown nodes q that share a cell with it, from the element matrices of
    its (up to 4) cells.  kx, ky: [ncy][ncx] cell arrays.  For checking single
    rows of grids too large to assemble."""
    Ex, Ey = q1_element_matrices(g.hx, g.hy)
    out: dict = {}
    for cj in (j - 1, j):
        if g.periodic_y:
            cj %= g.ncy
        elif cj < 0 or cj >= g.ncy:
            continue
        for ci in (i - 1, i):
            if ci < 0 or ci >= g.ncx:
                continue
            E = kx[cj, ci] * Ex + ky[cj, ci] * Ey
            nodes = _cell_nodes(g, ci, cj)
            p = nodes.index((j % g.ny if g.periodic_y else j, i))
            for q, (jq, iq) in enumerate(nodes):
                if iq < 1 or iq > g.nx - 2 or (not g.periodic_y and (jq < 1 or jq > g.ny - 2)):
                    continue
                out[(jq, iq)] = out.get((jq, iq), 0.0) + E[p, q]
    return out


def restriction(gf: Grid) -> sp.csr_matrix:
    """Full weighting R = (1/16)[1 2 1; 2 4 2; 1 2 1] from ``gf`` to ``gf.coarse()``
    on the unknowns (the restriction R_l^{l-1} of the multigrid algorithm)."""
    Rx = _fw_1d(gf.nx, False)
    Ry = _fw_1d(gf.ny, gf.periodic_y)
    return sp.kron(Ry, Rx).tocsr()


def prolongation(gf: Grid) -> sp.csr_matrix:
    """Bilinear interpolation P_{l-1}^l from ``gf.coarse()`` to ``gf``: P = 4 R^T
    (injection at coincident nodes, averages of 2 and of 4 elsewhere)."""
    return (4.0 * restriction(gf).T).tocsr()


# --------------------------------------------------------------------------- smoothers


def colour_sets(g: Grid, ncolours: int) -> list[np.ndarray]:
    """Unknown indices per colour, in sweep order.  2 colours: red = (i + j)
    even, then black.  4 colours: (i mod 2, j mod 2) in the order (0,0), (1,0),
    (0,1), (1,1).  i, j are stored level indices (i = 0 on the boundary)."""
    J, I = np.meshgrid(np.array(g.uy), np.array(g.ux), indexing="ij")
    I = I.reshape(-1)
    J = J.reshape(-1)
    if ncolours == 2:
        c = (I + J) % 2
        return [np.nonzero(c == 0)[0], np.nonzero(c == 1)[0]]
    if ncolours == 4:
        c = (I % 2) + 2 * (J % 2)
        return [np.nonzero(c == k)[0] for k in range(4)]
    raise ValueError("ncolours must be 2 or 4")


LINE_SMOOTHERS = ("tri_x", "tri_y", "adi", "gstri_x", "gstri_y", "gsadi")


def _unknown_ij(g: Grid) -> tuple[np.ndarray, np.ndarray]:
    """Stored (i, j) of every unknown, in unknown-vector order."""
    J, I = np.meshgrid(np.array(g.uy), np.array(g.ux), indexing="ij")
    return I.reshape(-1), J.reshape(-1)


def line_part(g: Grid, A, direction: str) -> sp.csr_matrix:
    """Tridiagonal preconditioner of the TRI smoothers ("The choice of C": D
    plus the first sub- and super-diagonals in the ordering that runs along the
    lines): the entries of A that couple an unknown with itself and with its
    two neighbours on the same grid line, lines along x (rows, "TRIx") or
    along y (columns, "TRIy"; the neighbours wrap across a periodic seam)."""
    I, J = _unknown_ij(g)
    a = sp.coo_matrix(A)
    r, c = a.row, a.col
    if direction == "x":
        keep = (J[r] == J[c]) & (np.abs(I[r] - I[c]) <= 1)
    elif direction == "y":
        dj = np.abs(J[r] - J[c])
        if g.periodic_y:
            dj = np.minimum(dj, g.ny - dj)
        keep = (I[r] == I[c]) & (dj <= 1)
    else:
        raise ValueError("direction must be 'x' or 'y'")
    return sp.csr_matrix((a.data[keep], (r[keep], c[keep])), shape=A.shape)


def line_colour_sets(g: Grid, direction: str) -> list[np.ndarray]:
    """Unknowns of the two zebra line colours, in sweep order: lines along x
    are rows j, lines along y columns i; colour 0 = even stored index, first."""
    I, J = _unknown_ij(g)
    key = J if direction == "x" else I
    return [np.nonzero(key % 2 == 0)[0], np.nonzero(key % 2 == 1)[0]]


def tri_step(A, T, x, b, omega):
    """Preconditioned Richardson with C = T (TRI, line Jacobi):
    x + omega T^{-1} (b - A x), every line solved exactly at once."""
    return x + omega * spla.spsolve(sp.csc_matrix(T), b - A @ x)


def line_gs_step(A, x, b, sets):
    """Gauss-Seidel over lines (GSTRI, omega = 1): for each line colour in
    turn, the lines of that colour are solved exactly with the latest values
    on the lines of the other colour (lines of one colour do not couple)."""
    x = x.copy()
    A = sp.csr_matrix(A)
    n = len(x)
    for s in sets:
        rest = np.setdiff1d(np.arange(n), s)
        rhs = b[s] - A[s][:, rest] @ x[rest]
        x[s] = spla.spsolve(sp.csc_matrix(A[s][:, s]), rhs)
    return x


def jacobi_step(A, diag, x, b, omega):
    """Preconditioned Richardson with C = D: x + omega D^{-1} (b - A x)."""
    return x + omega * (b - A @ x) / diag


def coloured_gs_step(A, diag, x, b, colours, omega=1.0):
    """One Gauss-Seidel step (C = D + omega L in colour order; omega = 1 is
    plain GS).  Nodes of one colour are not coupled to each other, so the
    update of a colour is x_c <- x_c + omega (b_c - (A x)_c) / d_c using the
    latest values of every other colour."""
    x = x.copy()
    for c in colours:
        r_c = b[c] - A[c, :] @ x
        x[c] = x[c] + omega * r_c / diag[c]
    return x


# --------------------------------------------------------------------------- hierarchy and cycle


@dataclass
class Options:
    cycle: str = "F"          # "F", "V" or "W"
    smoother: str = "rbgs"    # "jacobi", "rbgs" (2 colours), "gs4c" (4 colours), or one of LINE_SMOOTHERS
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8        # Jacobi and TRI / ADI damping
    sor: float = 1.0          # Gauss-Seidel / SOR factor in (0, 2) ("The choice of C": C = D + omega L); 1 = GS
    adaptive_omega: bool = False  # coarse-correction weight omega_l minimising the energy norm (else omega_l = 1)


@dataclass
class Hierarchy:
    grids: list
    A: list                   # sparse operator per level (FP64)
    R: list                   # restriction from level l to l+1
    P: list                   # prolongation from level l+1 to l
    diag: list
    colours: list
    chol: tuple = None        # Cholesky factor of the coarsest operator (FP64)
    opts: Options = field(default_factory=Options)
    lines: list = None        # line smoothers: per level {"Tx", "Ty", "sx", "sy"}

    @property
    def nlevels(self) -> int:
        return len(self.grids)

    def astype(self, dtype) -> "Hierarchy":
        """Copy whose level operators, transfers and vectors are in ``dtype``;
        the coarsest factor stays FP64."""
        lines = None
        if self.lines is not None:
            lines = [{"Tx": L["Tx"].astype(dtype), "Ty": L["Ty"].astype(dtype), "sx": L["sx"], "sy": L["sy"]}
                     for L in self.lines]
        return Hierarchy(self.grids, [a.astype(dtype) for a in self.A], [r.astype(dtype) for r in self.R],
                         [p.astype(dtype) for p in self.P], [d.astype(dtype) for d in self.diag],
                         self.colours, self.chol, self.opts, lines)


def build_hierarchy(g: Grid, A0: sp.spmatrix, opts: Options, levels: int = 0,
                    rediscretise=None) -> Hierarchy:
    """Level operators A_l (a1): ``rediscretise(grid)`` when given (5-point
    problems), else Galerkin A_{l+1} = R_l A_l P_l (9-point problems)."""
    grids = hierarchy_grids(g, levels)
    A = [A0.tocsr()]
    R, P = [], []
    for l in range(len(grids) - 1):
        R.append(restriction(grids[l]))
        P.append(prolongation(grids[l]))
        if rediscretise is not None:
            A.append(rediscretise(grids[l + 1]).tocsr())
        else:
            A.append((R[l] @ A[l] @ P[l]).tocsr())
    ncol = 0 if opts.smoother in LINE_SMOOTHERS else {"jacobi": 0, "rbgs": 2, "gs4c": 4}[opts.smoother]
    colours = [colour_sets(gl, ncol) if ncol else None for gl in grids]
    diag = [a.diagonal().copy() for a in A]
    chol = sla.cho_factor(A[-1].toarray(), lower=True)
    lines = None
    if opts.smoother in LINE_SMOOTHERS:
        lines = [{"Tx": line_part(gl, a, "x"), "Ty": line_part(gl, a, "y"), "sx": line_colour_sets(gl, "x"),
                  "sy": line_colour_sets(gl, "y")} for gl, a in zip(grids, A)]
    return Hierarchy(grids, A, R, P, diag, colours, chol, opts, lines)


def hierarchy_5pt(g: Grid, eps_x=1.0, eps_y=1.0, opts=None, levels=0, galerkin=False) -> Hierarchy:
    """5-point hierarchy: every level rediscretised (H = 2h), or with
    ``galerkin`` the coarse levels as R A P of the level above (9-point)."""
    opts = opts or Options()
    redisc = None if galerkin else (lambda gl: laplace5(gl, eps_x, eps_y))
    return build_hierarchy(g, laplace5(g, eps_x, eps_y), opts, levels, rediscretise=redisc)


def hierarchy_q1(g: Grid, kx, ky, opts=None, levels=0, separable=False, xs=None, ys=None) -> Hierarchy:
    """Q1 hierarchy: the finest operator assembled from cells (on the refined
    grid xs, ys when given), the coarse levels Galerkin R A P with the
    transfers of the logically equidistant grid."""
    opts = opts or Options(smoother="gs4c")
    if xs is not None or ys is not None:
        A0 = assemble_q1_graded(g, xs, ys, kx, ky)
    else:
        A0 = assemble_q1_separable(g, kx, ky) if separable else assemble_q1(g, kx, ky)
    return build_hierarchy(g, A0, opts, levels, rediscretise=None)


def line_smoothing_step(h: Hierarchy, l: int, x, g):
    """One step of a line smoother on level l (an ADI or GSADI step is the
    x-line half followed by the y-line half)."""
    o, A, L = h.opts, h.A[l], h.lines[l]
    if o.smoother in ("tri_x", "adi"):
        x = tri_step(A, L["Tx"], x, g, o.omega)
    if o.smoother in ("tri_y", "adi"):
        x = tri_step(A, L["Ty"], x, g, o.omega)
    if o.smoother in ("gstri_x", "gsadi"):
        x = line_gs_step(A, x, g, L["sx"])
    if o.smoother in ("gstri_y", "gsadi"):
        x = line_gs_step(A, x, g, L["sy"])
    return x


def smooth(h: Hierarchy, l: int, x, g, steps: int):
    o = h.opts
    for _ in range(steps):
        if o.smoother == "jacobi":
            x = jacobi_step(h.A[l], h.diag[l], x, g, o.omega)
        elif o.smoother in LINE_SMOOTHERS:
            x = line_smoothing_step(h, l, x, g)
        else:
            x = coloured_gs_step(h.A[l], h.diag[l], x, g, h.colours[l], o.sor)
    return x


def coarse_solve(h: Hierarchy, g):
    """Exact solve A_1^{-1} g on the coarsest level with the FP64 Cholesky factor."""
    out = sla.cho_solve(h.chol, np.asarray(g, dtype=np.float64))
    return out.astype(g.dtype)


def coarse_correction(h: Hierarchy, l: int, x, g, kind: str):
    """Correction to add on level l (before the weight omega_l): the defect of
    x, restricted by full weighting, is the right-hand side of the next
    coarser level, whose equation is then solved approximately from zero by
    the recursive calls the cycle kind prescribes; returns the prolonged
    result (an F-cycle spends one F-cycle and then one V-cycle on the coarse
    problem, a V-cycle one V-cycle, a W-cycle two W-cycles, the second one
    continuing from the first)."""
    gc = h.R[l] @ (g - h.A[l] @ x)
    e = np.zeros_like(gc)
    calls = {"F": ("F", "V"), "W": ("W", "W"), "V": ("V",)}[kind]
    for k in calls:
        e = mg_cycle(h, l + 1, e, gc, k)
    return h.P[l] @ e


def energy_weight(h: Hierarchy, l: int, x, g, pe) -> float:
    """The coarse-correction weight that minimises the A-norm of the error of
    x + w pe along the prolonged correction pe (the adaptive choice the paper
    allows for omega_l): w = (d, pe) / (A pe, pe) with d = g - A x the defect.
    A zero correction gets weight 1."""
    d = g - h.A[l] @ x
    ape = h.A[l] @ pe
    den = float(np.dot(ape, pe))
    return float(np.dot(d, pe)) / den if den != 0.0 else 1.0


def mg_cycle(h: Hierarchy, l: int, x, g, kind: str = "F"):
    """One cycle of the recursive multigrid algorithm of "The Multigrid
    Technique" on level l (0 = finest; the paper numbers its levels upwards
    from the coarsest): nu_pre smoothing steps, the coarse-grid correction of
    :func:`coarse_correction` added with weight omega_l (1, or the
    energy-minimising weight of :func:`energy_weight` when
    ``opts.adaptive_omega`` is set), then nu_post smoothing steps.  On the
    coarsest level the equation is solved exactly."""
    if l == h.nlevels - 1:
        return coarse_solve(h, g)
    o = h.opts
    x = smooth(h, l, x, g, o.nu_pre)
    pe = coarse_correction(h, l, x, g, kind)
    w = energy_weight(h, l, x, g, pe) if o.adaptive_omega else 1.0
    x = x + w * pe if o.adaptive_omega else x + pe
    return smooth(h, l, x, g, o.nu_post)


def nested_start(h: Hierarchy, b, kind: str = None):
    """Start vector by nested iteration (section "Start-Vector Choice": the
    solution starts on the coarsest grid and is carried level by level to the
    finest one): the right-hand side is
    restricted to every level (b_{l+1} = R b_l), the coarsest problem is solved
    exactly, and on each finer level l >= 1 the prolonged coarser result is
    improved by one cycle of the hierarchy's kind with rhs b_l; the finest
    start is the prolongation of level 1's result."""
    kind = kind or h.opts.cycle
    bs = [np.asarray(b, dtype=np.float64)]
    for l in range(h.nlevels - 1):
        bs.append(h.R[l] @ bs[-1])
    x = coarse_solve(h, bs[-1])
    for l in range(h.nlevels - 2, 0, -1):
        x = mg_cycle(h, l, h.P[l] @ x, bs[l], kind)
    return h.P[0] @ x if h.nlevels > 1 else x


def residual_norm(h: Hierarchy, b, x) -> float:
    """2-norm of b - A x over the unknowns of the finest level (FP64)."""
    r = np.asarray(b, dtype=np.float64) - h.A[0] @ np.asarray(x, dtype=np.float64)
    return float(np.sqrt(np.dot(r, r)))


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    cycles: int
    history: list


def solve(h: Hierarchy, b, x0, tol: float, max_cycles: int) -> SolveResult:
    """Cycle until ||b - A x_k|| <= tol ||b - A x_0|| (relative residual), or
    max_cycles, or divergence (non-finite or > 1e6 r0).  Vectors are unknown
    vectors (see Grid.pack)."""
    kind = h.opts.cycle
    x = np.asarray(x0, dtype=np.float64).copy()
    b = np.asarray(b, dtype=np.float64)
    r0 = residual_norm(h, b, x)
    hist = [r0]
    if r0 == 0.0:
        return SolveResult(x, OK, 0, hist)
    status = NOT_CONVERGED
    k = 0
    while k < max_cycles:
        x = mg_cycle(h, 0, x, b, kind)
        k += 1
        r = residual_norm(h, b, x)
        hist.append(r)
        if r <= tol * r0:
            status = OK
            break
        if not math.isfinite(r) or r > DIVERGENCE_FACTOR * r0:
            status = DIVERGED
            break
    return SolveResult(x, status, k, hist)


def solve_mixed(h: Hierarchy, b, x0, tol: float, max_cycles: int, h32: Hierarchy = None,
                inner: int = 1) -> SolveResult:
    """Defect correction: FP64 residual r = b - A x and its norm; ``inner``
    FP32 cycles for A e = (float) r from e = 0; x += (double) e.  Stop as in
    :func:`solve`; ``cycles`` counts the outer steps.  The inner hierarchy
    ``h32`` (default: ``h`` in FP32) sets the inner precision; r is rounded to
    its type."""
    h32 = h32 or h.astype(np.float32)
    inner_type = h32.A[0].dtype
    kind = h.opts.cycle
    x = np.asarray(x0, dtype=np.float64).copy()
    b = np.asarray(b, dtype=np.float64)
    r = b - h.A[0] @ x
    r0 = float(np.sqrt(np.dot(r, r)))
    hist = [r0]
    if r0 == 0.0:
        return SolveResult(x, OK, 0, hist)
    status = NOT_CONVERGED
    k = 0
    while k < max_cycles:
        r32 = r.astype(inner_type)
        e = np.zeros_like(r32)
        for _ in range(inner):
            e = mg_cycle(h32, 0, e, r32, kind)
        x = x + e.astype(np.float64)
        k += 1
        r = b - h.A[0] @ x
        rn = float(np.sqrt(np.dot(r, r)))
        hist.append(rn)
        if rn <= tol * r0:
            status = OK
            break
        if not math.isfinite(rn) or rn > DIVERGENCE_FACTOR * r0:
            status = DIVERGED
            break
    return SolveResult(x, status, k, hist)


# --------------------------------------------------------------------------- adjoint


def q1_coeff_grad(g: Grid, u_stored: np.ndarray, lam_stored: np.ndarray, part: str = "a") -> np.ndarray:
    """Per-cell derivative of L(a) = 1/2 ||u(a) - u*||^2 with A(a) u = f:
    dL/da_c = -lam_e^T (dA/da_c) u_e with lam = A^{-T} (u - u*).  ``part`` = "a"
    (kx = ky = a), "kx" or "ky".  u, lam are stored arrays with zero boundary."""
    Ex, Ey = q1_element_matrices(g.hx, g.hy)
    K = {"a": Ex + Ey, "kx": Ex, "ky": Ey}[part]
    u = np.asarray(u_stored, dtype=np.float64).reshape(g.ny, g.nx)
    lam = np.asarray(lam_stored, dtype=np.float64).reshape(g.ny, g.nx)
    out = np.zeros((g.ncy, g.ncx))
    for cj in range(g.ncy):
        for ci in range(g.ncx):
            nodes = _cell_nodes(g, ci, cj)
            ue = np.array([u[j, i] for j, i in nodes])
            le = np.array([lam[j, i] for j, i in nodes])
            out[cj, ci] = -le @ K @ ue
    return out


def q1_coeff_grad_vectorised(g: Grid, u_stored: np.ndarray, lam_stored: np.ndarray, part: str = "a") -> np.ndarray:
    """:func:`q1_coeff_grad` with the cell loop written as array slices (same
    formula, same element matrix); for grids too large for the Python loop."""
    Ex, Ey = q1_element_matrices(g.hx, g.hy)
    K = {"a": Ex + Ey, "kx": Ex, "ky": Ey}[part]
    u = np.asarray(u_stored, dtype=np.float64).reshape(g.ny, g.nx)
    lam = np.asarray(lam_stored, dtype=np.float64).reshape(g.ny, g.nx)
    if g.periodic_y:
        u = np.vstack([u, u[:1]])
        lam = np.vstack([lam, lam[:1]])
    ue = [u[b:b + g.ncy, a:a + g.ncx] for b in range(2) for a in range(2)]
    le = [lam[b:b + g.ncy, a:a + g.ncx] for b in range(2) for a in range(2)]
    out = np.zeros((g.ncy, g.ncx))
    for p in range(4):
        for q in range(4):
            if K[p, q] != 0.0:
                out -= le[p] * K[p, q] * ue[q]
    return out


def adjoint_gradient(g: Grid, a: np.ndarray, f_stored: np.ndarray, u_target_stored: np.ndarray):
    """Exact (direct-solve) gradient of L = 1/2 sum_interior (u - u*)^2 for the
    isotropic Q1 problem -div(a grad u) = f with lumped right-hand side b = f.
    Returns (u, lam, dL/da per cell, dL/df = lam), arrays stored [ny][nx]."""
    A = assemble_q1(g, a, a) if g.n_unknowns <= 40000 else None
    if A is None:
        raise ValueError("adjoint_gradient uses element-by-element assembly; grid too large")
    b = g.pack(f_stored)
    u = spla.spsolve(A.tocsc(), b)
    lam = spla.spsolve(A.T.tocsc(), u - g.pack(u_target_stored))
    u_s, lam_s = g.unpack(u), g.unpack(lam)
    return u_s, lam_s, q1_coeff_grad(g, u_s, lam_s, "a"), lam_s


def cycle_matrix(h: Hierarchy, kind: str = "F") -> np.ndarray:
    """Dense iteration matrix M of one cycle with b = 0 (x_{k+1} = M x_k),
    built by applying the cycle to unit vectors (tiny grids only)."""
    n = h.grids[0].n_unknowns
    M = np.zeros((n, n))
    zero = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = mg_cycle(h, 0, e, zero, kind)
    return M
