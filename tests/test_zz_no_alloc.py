"""mg_residual_noalloc (no handle, no device allocation: the library's static
scratch) against mg_residual on a handle for the same grid and operator,
called twice in a row with the second input smaller; the scratch keeps the
first call's contents, so the second call checks that everything it needs
is rewritten."""

import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mg():
    from paper_0805_3041_amd import mg
    return mg


def _inputs(nx, ny, seed, periodic_y=False):
    rhs = torch.tensor(W.normal_field(nx, ny, seed, periodic_y), device="cuda")
    x = torch.tensor(np.random.default_rng(seed + 1).uniform(-1, 1, (ny, nx)), device="cuda")
    x[:, 0] = 5.0   # boundary values are read as zero by both calls
    x[:, -1] = 5.0
    if not periodic_y:
        x[0, :] = 5.0
        x[-1, :] = 5.0
    return rhs, x


def _both(solver, rhs, x):
    """(r, norm) from the handle's mg_residual and from mg_residual_noalloc."""
    mg = _mg()
    r_h = torch.full_like(x, 9.0)
    n_h = solver.residual(rhs, x, r_h)
    r_n = torch.full_like(x, 7.0)  # stale values: the call must write every node
    n_n = mg.mg_residual_noalloc(solver.grid, solver.coeffs, rhs, x, r_n)
    torch.cuda.synchronize()
    return r_h.cpu().numpy(), n_h, r_n.cpu().numpy(), n_n


def test_const5_two_calls_second_smaller_bitwise():
    mg = _mg()
    for nx, ny, eps in ((257, 193, 0.3), (65, 33, 2.0)):
        s = mg.Solver(nx, ny, eps_x=eps)
        try:
            rhs, x = _inputs(nx, ny, 3)
            r_h, n_h, r_n, n_n = _both(s, rhs, x)
        finally:
            s.close()
        np.testing.assert_array_equal(r_n, r_h)
        assert n_n == n_h
        assert np.all(r_n[:, 0] == 0) and np.all(r_n[0, :] == 0)


def test_cell9_two_calls_second_smaller():
    """257^2 cell coefficients: the handle's finest level forms its couplings
    from the cells as the no-alloc call does (bit for bit); then a 65^2 grid,
    whose handle reads assembled bands (equal up to rounding, 1e-13 of the
    largest entry), and a periodic annulus with 1-D coefficients."""
    mg = _mg()
    for n in (257, 65):
        a = torch.tensor(np.exp(W.gaussian_random_field(n - 1, 5)), device="cuda")
        s = mg.Solver(n, n, kx=a, ky=a, smoother="gs4c")
        try:
            rhs, x = _inputs(n, n, 4)
            r_h, n_h, r_n, n_n = _both(s, rhs, x)
        finally:
            s.close()
        scale = np.abs(r_h).max()
        if n == 257:
            np.testing.assert_array_equal(r_n, r_h)
            assert n_n == n_h
        else:
            assert np.abs(r_n - r_h).max() <= 1e-13 * scale
            assert abs(n_n - n_h) <= 1e-13 * n_h
        assert np.all(r_n[:, 0] == 0) and np.all(r_n[:, -1] == 0) and np.all(r_n[-1, :] == 0)
    nx, ny = 129, 128
    kx, ky = W.annulus_cell_coefficients(nx)
    s = mg.Solver(nx, ny, periodic_y=True, kx=torch.tensor(kx, device="cuda"), ky=torch.tensor(ky, device="cuda"),
                  kx_1d_along_x=True, smoother="gs4c")
    try:
        rhs, x = _inputs(nx, ny, 5, periodic_y=True)
        r_h, n_h, r_n, n_n = _both(s, rhs, x)
    finally:
        s.close()
    assert np.abs(r_n - r_h).max() <= 1e-13 * np.abs(r_h).max()
    assert abs(n_n - n_h) <= 1e-13 * n_h


def test_rejects_sizes_beyond_the_scratch_and_bad_arguments():
    mg = _mg()
    lib = mg.load_library()
    rhs = torch.zeros((5, 5), dtype=torch.float64, device="cuda")
    nrm = ctypes.c_double()
    c5 = mg.mg_coeffs(mg.MG_COEF_CONST5, 1.0, 1.0, None, None, 0)
    big = mg.mg_grid(65539, 3, 0, 0, 1.0, 1.0)
    s = lib.mg_residual_noalloc(ctypes.byref(big), ctypes.byref(c5), mg._ptr(rhs), mg._ptr(rhs), None,
                                ctypes.byref(nrm), None)
    assert s == mg.MG_EINVAL and "65537" in mg.last_error(None)
    g = mg.mg_grid(5, 5, 0, 0, 1.0, 1.0)
    bad = mg.mg_coeffs(mg.MG_COEF_CELL9, 0.0, 0.0, None, None, 0)
    assert lib.mg_residual_noalloc(ctypes.byref(g), ctypes.byref(bad), mg._ptr(rhs), mg._ptr(rhs), None,
                                   ctypes.byref(nrm), None) == mg.MG_EINVAL
    assert lib.mg_residual_noalloc(ctypes.byref(g), ctypes.byref(c5), None, mg._ptr(rhs), None,
                                   ctypes.byref(nrm), None) == mg.MG_EINVAL
