"""Seeded synthetic inputs for the multigrid workloads.

This module holds input generation only (grids' node coordinates, seeded random
right-hand sides and start vectors, coefficient fields of the test problems).
It contains none of the solver's arithmetic: no stencil, smoother, transfer
operator or cycle.  Both the GPU tests/bench and the CPU oracle's tests take
their inputs from here.

Workloads (the paper prints no grid sizes; these are synthetic stand-ins with
the structure the paper describes):

* ``poisson65``  : 65 x 65 unit square, zero Dirichlet, 5-point, Jacobi F-cycle.
* ``aniso1025``  : 1025 x 1025, -(eps u_xx + u_yy), eps in {1, 1e-1, 1e-2, 1e-3},
                   red-black Gauss-Seidel, 1-4 smoothing steps, zero or U[-1, 1] start.
* ``annulus``    : r in [0.5, 1], theta periodic, mapped to the unit square,
                   4097 (radial, Dirichlet) x 4096 (angular, periodic) nodes, Q1.
* ``batch256``   : 256 problems, n drawn from {129, 257, 513, 1025}, eps log-uniform.
* ``grf2049``    : -div(a grad u) = f on 2049^2 nodes, a = exp(GRF).
"""

from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------- coordinates


def node_coords(nx: int, ny: int, periodic_y: bool = False, lx: float = 1.0, ly: float = 1.0):
    """(X, Y) arrays [ny][nx] of node coordinates."""
    x = np.arange(nx) * (lx / (nx - 1))
    y = np.arange(ny) * (ly / ny if periodic_y else ly / (ny - 1))
    Y, X = np.meshgrid(y, x, indexing="ij")
    return X, Y


def zero_boundary(u: np.ndarray, periodic_y: bool = False) -> np.ndarray:
    u = np.array(u, dtype=np.float64, copy=True)
    u[:, 0] = 0.0
    u[:, -1] = 0.0
    if not periodic_y:
        u[0, :] = 0.0
        u[-1, :] = 0.0
    return u


# --------------------------------------------------------------------------- generic draws


def normal_field(nx: int, ny: int, seed: int, periodic_y: bool = False) -> np.ndarray:
    """N(0, 1) values at every stored node (PCG64 ``default_rng(seed)``), boundary zeroed."""
    rng = np.random.default_rng(seed)
    return zero_boundary(rng.standard_normal((ny, nx)), periodic_y)


def uniform_field(nx: int, ny: int, seed: int, periodic_y: bool = False) -> np.ndarray:
    """U[-1, 1] values at every stored node, boundary zeroed (random start vector)."""
    rng = np.random.default_rng(seed)
    return zero_boundary(rng.uniform(-1.0, 1.0, (ny, nx)), periodic_y)


# --------------------------------------------------------------------------- square problems


def manufactured_sine(n: int, eps: float = 1.0):
    """u = sin(pi x) sin(pi y) and f = (1 + eps) pi^2 u for -(eps u_xx + u_yy) = f."""
    X, Y = node_coords(n, n)
    u = np.sin(np.pi * X) * np.sin(np.pi * Y)
    return zero_boundary((1.0 + eps) * np.pi**2 * u), zero_boundary(u)


ANISO_EPS = (1.0, 1e-1, 1e-2, 1e-3)


def aniso_rhs(n: int = 1025, seed: int = 2) -> np.ndarray:
    return normal_field(n, n, seed)


def aniso_x0(n: int = 1025, kind: str = "zero", seed: int = 1) -> np.ndarray:
    if kind == "zero":
        return np.zeros((n, n))
    return uniform_field(n, n, seed)


# --------------------------------------------------------------------------- annulus


ANNULUS_R0, ANNULUS_R1 = 0.5, 1.0


def graded_nodes(n: int, a: float = 0.0, length: float = 1.0) -> np.ndarray:
    """n node coordinates on [0, length], refined toward 0 for a > 0 (toward
    `length` for a < 0): x = length (e^(a xi) - 1) / (e^a - 1) at equidistant
    xi in [0, 1]; a = 0 gives the equidistant grid.  The spacing ratio between
    the last and the first cell is about e^a."""
    xi = np.linspace(0.0, 1.0, n)
    if a == 0.0:
        return length * xi
    x = length * np.expm1(a * xi) / np.expm1(a)
    x[0], x[-1] = 0.0, length
    return x


def lumped_rhs(f: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Right-hand side of the Q1 operator on a refined tensor grid (Dirichlet
    both ways) with a lumped mass: b = f times the node's dual area
    (half-cells on each side), over hx0 hy0 of the equidistant grid of the
    same extent; zero at boundary nodes."""
    hx, hy = np.diff(xs), np.diff(ys)
    dx = np.zeros(len(xs))
    dy = np.zeros(len(ys))
    dx[1:-1] = 0.5 * (hx[:-1] + hx[1:])
    dy[1:-1] = 0.5 * (hy[:-1] + hy[1:])
    hx0 = (xs[-1] - xs[0]) / (len(xs) - 1)
    hy0 = (ys[-1] - ys[0]) / (len(ys) - 1)
    return np.asarray(f, dtype=np.float64) * np.outer(dy, dx) / (hx0 * hy0)


def annulus_cell_coefficients(nx: int):
    """Per radial cell (length nx - 1) coefficients of the annulus mapped to the
    unit square: with r = 0.5 + 0.5 xi and theta = 2 pi eta, the weak form of
    -Laplace(u) in polar coordinates, int (u_r v_r + u_theta v_theta / r^2) r dr dtheta,
    becomes int (4 pi r u_xi v_xi + u_eta v_eta / (4 pi r)) dxi deta.  The cell
    value uses the midpoint radius."""
    hx = 1.0 / (nx - 1)
    xi_c = (np.arange(nx - 1) + 0.5) * hx
    r_c = ANNULUS_R0 + (ANNULUS_R1 - ANNULUS_R0) * xi_c
    kx = 4.0 * np.pi * r_c
    ky = 1.0 / (4.0 * np.pi * r_c)
    return kx, ky


# Spherical coordinates (r, theta) of an axisymmetric shell section, away
# from the axis: r in [0.5, 1], theta in [0.1 pi, 0.9 pi].
SPHERE_R0, SPHERE_R1 = 0.5, 1.0
SPHERE_T0, SPHERE_T1 = 0.1 * np.pi, 0.9 * np.pi


def sphere_cell_coefficients(nx: int, ny: int):
    """Per-cell ([ny-1][nx-1]) coefficients of -Laplace(u) in spherical
    coordinates (axisymmetric), whose weak form carries the volume weight
    r^2 sin(theta): int (r^2 sin(theta) u_r v_r + sin(theta) u_theta v_theta)
    dr dtheta.  Mapped to the unit square (r = R0 + Lr xi, theta = T0 +
    Lt eta) it becomes int (kx u_xi v_xi + ky u_eta v_eta) dxi deta with
    kx = r^2 sin(theta) Lt / Lr and ky = sin(theta) Lr / Lt, evaluated at
    the cell midpoint; both vary over the cells in both directions."""
    lr, lt = SPHERE_R1 - SPHERE_R0, SPHERE_T1 - SPHERE_T0
    xi = (np.arange(nx - 1) + 0.5) / (nx - 1)
    eta = (np.arange(ny - 1) + 0.5) / (ny - 1)
    R, T = np.meshgrid(SPHERE_R0 + lr * xi, SPHERE_T0 + lt * eta)
    kx = R * R * np.sin(T) * lt / lr
    ky = np.sin(T) * lr / lt
    return np.ascontiguousarray(kx), np.ascontiguousarray(ky)


def sphere_manufactured(n: int):
    """u = sin(pi xi) sin(pi eta) (zero on the boundary) and the nodal values
    of -d/dxi (kx u_xi) - d/deta (ky u_eta) for the continuous kx, ky of
    sphere_cell_coefficients, written out by the product rule; returns
    (f, u) as [n][n] arrays."""
    lr, lt = SPHERE_R1 - SPHERE_R0, SPHERE_T1 - SPHERE_T0
    X, Y = node_coords(n, n)
    r, t = SPHERE_R0 + lr * X, SPHERE_T0 + lt * Y
    sx, cx = np.sin(np.pi * X), np.cos(np.pi * X)
    sy, cy = np.sin(np.pi * Y), np.cos(np.pi * Y)
    u = sx * sy
    # d/dxi (kx u_xi), kx = r^2 sin(t) lt/lr, dr/dxi = lr
    d_x = (lt / lr) * np.sin(t) * sy * np.pi * (2.0 * r * lr * cx - r * r * np.pi * sx)
    # d/deta (ky u_eta), ky = sin(t) lr/lt, dt/deta = lt
    d_y = (lr / lt) * sx * np.pi * (lt * np.cos(t) * cy - np.pi * np.sin(t) * sy)
    return zero_boundary(-(d_x + d_y)), zero_boundary(u)


def annulus_radius(nx: int, ny: int) -> np.ndarray:
    X, _ = node_coords(nx, ny, periodic_y=True)
    return ANNULUS_R0 + (ANNULUS_R1 - ANNULUS_R0) * X


def annulus_rhs_from_f(f: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """Lumped right-hand side b_i = pi r_i f_i: the polar area element r dr dtheta
    = pi r dxi deta of the mapping, divided by the cell area (FD scaling)."""
    return zero_boundary(np.pi * annulus_radius(nx, ny) * f, periodic_y=True)


def annulus_manufactured(nx: int, ny: int):
    """u = sin(2 pi (r - 1/2)) cos(theta) and f = -Laplace(u) in polar form:
    f = (4 pi^2 s - 2 pi c / r + s / r^2) cos(theta) with s, c = sin, cos of 2 pi (r - 1/2).
    Returns (b, u) as stored arrays."""
    X, Y = node_coords(nx, ny, periodic_y=True)
    r = ANNULUS_R0 + (ANNULUS_R1 - ANNULUS_R0) * X
    th = 2.0 * np.pi * Y
    s = np.sin(2.0 * np.pi * (r - 0.5))
    c = np.cos(2.0 * np.pi * (r - 0.5))
    u = s * np.cos(th)
    f = (4.0 * np.pi**2 * s - 2.0 * np.pi * c / r + s / r**2) * np.cos(th)
    return annulus_rhs_from_f(f, nx, ny), zero_boundary(u, periodic_y=True)


def annulus_rhs(nx: int = 4097, ny: int = 4096, seed: int = 3) -> np.ndarray:
    return normal_field(nx, ny, seed, periodic_y=True)


# --------------------------------------------------------------------------- Gaussian random field


def gaussian_random_field(ncells: int, seed: int, length: float = 0.1, sigma: float = 1.0) -> np.ndarray:
    """Stationary Gaussian field with covariance sigma^2 exp(-d^2 / (2 length^2)) at
    the ncells^2 cell centres of [0, 1]^2, by circulant embedding (Dietrich and
    Newsam, 1997): the covariance is sampled on a periodic 2 ncells grid over
    [0, 2]^2, its FFT gives the circulant eigenvalues, and white noise filtered by
    their square roots has that covariance.  The doubled period keeps the wrap
    far outside the correlation length.  Returns [ncells][ncells]."""
    m = 2 * ncells
    h = 1.0 / ncells
    k = np.arange(m)
    d1 = np.minimum(k, m - k) * h
    D2 = d1[:, None] ** 2 + d1[None, :] ** 2
    c = sigma**2 * np.exp(-D2 / (2.0 * length**2))
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((m, m))
    g = np.fft.ifft2(np.fft.fft2(w) * np.sqrt(lam)).real
    return np.ascontiguousarray(g[:ncells, :ncells])


def grf_problem(n: int = 2049, seed: int = 5):
    """a = exp(g) per cell, f = 2 pi^2 sin(pi x) sin(pi y), u* = sin(pi x) sin(pi y)."""
    a = np.exp(gaussian_random_field(n - 1, seed))
    f, ustar = manufactured_sine(n, 1.0)
    return a, f, ustar


# --------------------------------------------------------------------------- batch


BATCH_SIZES = (129, 257, 513, 1025)


def batch_problems(nprob: int = 256, seed: int = 4, sizes=BATCH_SIZES):
    """Sizes drawn uniformly from ``sizes`` and eps = 10^U(-3, 0), one generator
    seeded with ``seed``; rhs of problem i is N(0, 1) with seed 1000 + i."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=nprob)
    eps = 10.0 ** rng.uniform(-3.0, 0.0, size=nprob)
    return [int(n) for n in ns], [float(e) for e in eps]


def batch_rhs(n: int, i: int) -> np.ndarray:
    return normal_field(n, n, 1000 + i)


def expected_unknowns(sizes=BATCH_SIZES, nprob: int = 256) -> float:
    return nprob * float(np.mean([(n - 2) ** 2 for n in sizes]))


def log_uniform(lo: float, hi: float, u: float) -> float:
    return 10.0 ** (math.log10(lo) + u * (math.log10(hi) - math.log10(lo)))
