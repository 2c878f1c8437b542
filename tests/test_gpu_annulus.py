"""Polar annulus mapped to the unit square (Q1, kx = 4 pi r, ky = 1/(4 pi r),
theta periodic), four-colour Gauss-Seidel F-cycle: parity with the oracle per
cycle at 1025 x 1024, and at the full 4097 x 4096 grid (16.8M unknowns)
properties the oracle can check row by row."""

import math

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W
from tests.problems import Problem

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _mg():
    from paper_0805_3041_amd import mg
    return mg


def _solver(n, precision="fp64"):
    mg = _mg()
    kx, ky = W.annulus_cell_coefficients(n)
    return mg.Solver(n, n - 1, periodic_y=True, kx=torch.tensor(kx, device="cuda"),
                     ky=torch.tensor(ky, device="cuda"), kx_1d_along_x=True, smoother="gs4c",
                     precision=precision)


def test_annulus1025_per_cycle_parity():
    from tests.test_gpu_parity import check_parity
    n = 1025
    p = Problem(n, n - 1, periodic_y=True, q1="annulus", smoother="gs4c")
    check_parity(p, W.annulus_rhs(n, n - 1, 3), np.zeros((n - 1, n)), 2)


def test_annulus4097_full_size_mixed_and_fp64():
    """Mixed and FP64 solves reach 1e-10; their residuals, recomputed row by row by
    the oracle at 4000 sampled nodes, match the library's; cycle counts agree within 2."""
    mg = _mg()
    n, ny = 4097, 4096
    rhs = torch.tensor(W.annulus_rhs(n, ny, 3), device="cuda")
    out = {}
    for prec in ("mixed", "fp64"):
        s = _solver(n, prec)
        x = torch.zeros((ny, n), dtype=torch.float64, device="cuda")
        info = s.solve(rhs, x, 1e-10, 400, history=False)
        r = torch.zeros_like(x)
        rn = s.residual(rhs, x, r)
        s.close()
        assert info.status == mg.MG_OK, (prec, info)
        assert rn <= 1.05e-10 * info.res0
        out[prec] = (info, x.cpu().numpy(), r.cpu().numpy())
    im, xm, rm = out["mixed"]
    i64, x64, r64 = out["fp64"]
    assert im.cycles <= i64.cycles + 2
    # oracle rows at sampled nodes
    g = O.Grid(n, ny, periodic_y=True)
    kx, ky = W.annulus_cell_coefficients(n)
    KX = np.broadcast_to(kx, (g.ncy, g.ncx))
    KY = np.broadcast_to(ky, (g.ncy, g.ncx))
    b = W.annulus_rhs(n, ny, 3)
    rng = np.random.default_rng(51)
    scale = np.abs(b).max()
    for x, r in ((xm, rm), (x64, r64)):
        for _ in range(4000):
            i = int(rng.integers(1, n - 1))
            j = int(rng.integers(0, ny))
            row = O.q1_row(g, KX, KY, i, j)
            ro = b[j, i] - sum(v * x[jq, iq] for (jq, iq), v in row.items())
            assert abs(ro - r[j, i]) <= 1e-9 * scale, (i, j, ro, r[j, i])
    # both solutions satisfy the same discrete system to 1e-10: they differ by at
    # most kappa * 2e-10 relative; the measured difference is reported here
    diff = np.abs(xm - x64).max() / np.abs(x64).max()
    assert diff < 1e-5, diff


def test_annulus_manufactured_second_order_to_full_size():
    """Manufactured u = sin(2 pi (r - 1/2)) cos(theta): the nodal max error of the
    GPU solution falls by 4 +- 0.4 per refinement up to 4097 x 4096."""
    errs = []
    for n in (1025, 2049, 4097):
        s = _solver(n, "fp64")
        b, u = W.annulus_manufactured(n, n - 1)
        x = torch.zeros((n - 1, n), dtype=torch.float64, device="cuda")
        # smooth right-hand side: the FP64 residual floor is near 1e-9 at h = 1/4096
        info = s.solve(torch.tensor(b, device="cuda"), x, 1e-8, 400, history=False)
        s.close()
        assert info.status == _mg().MG_OK
        errs.append(np.abs(x.cpu().numpy() - u).max())
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(abs(q - 4.0) < 0.4 for q in ratios), (errs, ratios)
