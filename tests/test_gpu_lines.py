"""GPU parity of the line smoothers (TRI, ADI, GSTRI, GSADI): the library's
line sweeps (cyclic reduction in LDS, one workgroup per line; one thread per
line with Thomas factors from setup for lines too long for LDS) against the
oracle's sparse line solves on the same seeded inputs, per cycle to 1e-12
relative max-norm in FP64; cycle counts to tolerance equal; the mixed form
reaches the tolerance; unsupported combinations are rejected."""

import numpy as np
import pytest

import workloads as W
from tests.problems import Problem
from tests.test_gpu_parity import check_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LINE_SMOOTHERS = ["tri_x", "tri_y", "adi", "gstri_x", "gstri_y", "gsadi"]


def _mg():
    from paper_0805_3041_amd import mg
    return mg


@pytest.mark.parametrize("smoother", LINE_SMOOTHERS)
@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-3])
def test_aniso65_per_cycle(smoother, eps):
    p = Problem(65, 65, eps=eps, smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(65, 65, 2), W.uniform_field(65, 65, 1), 4)


@pytest.mark.parametrize("smoother", ["adi", "gsadi"])
def test_ragged_rectangular_grid(smoother):
    """97 x 49 nodes: lines of different lengths in x and y, several
    workgroups of lines, ragged last workgroup."""
    p = Problem(97, 49, eps=0.05, smoother=smoother, omega=0.9)
    check_parity(p, W.normal_field(97, 49, 2), np.zeros((49, 97)), 3)


@pytest.mark.parametrize("smoother", ["tri_x", "gstri_x"])
def test_periodic_annulus_x_lines(smoother):
    """Lines along x on the periodic annulus (1-D bands, 9-point): the off-line
    couplings wrap across the seam."""
    p = Problem(65, 64, periodic_y=True, q1="annulus", smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(65, 64, 3, True), np.zeros((64, 65)), 3)


@pytest.mark.parametrize("smoother", ["adi", "gsadi", "gstri_y"])
def test_variable_q1_per_cycle(smoother):
    """2-D bands (Gaussian-random-field coefficient): line couplings and the
    six off-line couplings from the Galerkin bands of every level."""
    p = Problem(65, 65, q1="grf", smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(65, 65, 4), np.zeros((65, 65)), 3)


@pytest.mark.parametrize("smoother", ["tri_y", "gstri_y", "gsadi"])
def test_cycles_to_tolerance_match_oracle(smoother):
    from oracle import mg_oracle as O
    p = Problem(129, 129, eps=1e-3, smoother=smoother, omega=0.8)
    g = p.grid()
    rhs = W.normal_field(129, 129, 2)
    ro = O.solve(p.oracle(), g.pack(rhs), np.zeros(g.n_unknowns), 1e-10, 100)
    s = p.solver()
    try:
        x = torch.zeros((129, 129), dtype=torch.float64, device="cuda")
        info = s.solve(torch.tensor(rhs, device="cuda"), x, tol=1e-10, max_cycles=100)
    finally:
        s.close()
    assert ro.status == O.OK and info.status == 0
    assert info.cycles == ro.cycles
    assert info.cycles <= 12


@pytest.mark.parametrize("smoother", ["gstri_y", "adi"])
def test_mixed_precision_reaches_tolerance(smoother):
    """FP32 inner cycles with line sweeps inside the FP64 defect correction:
    the oracle's FP64 residual of the GPU result is below the tolerance."""
    from oracle import mg_oracle as O
    p = Problem(257, 257, eps=1e-3, smoother=smoother, omega=0.8)
    g = p.grid()
    rhs = W.normal_field(257, 257, 2)
    s = p.solver(precision="mixed")
    try:
        x = torch.zeros((257, 257), dtype=torch.float64, device="cuda")
        info = s.solve(torch.tensor(rhs, device="cuda"), x, tol=1e-10, max_cycles=60)
    finally:
        s.close()
    assert info.status == 0
    h = p.oracle()
    b = g.pack(rhs)
    rel = O.residual_norm(h, b, g.pack(x.cpu().numpy())) / O.residual_norm(h, b, np.zeros_like(b))
    assert rel <= 1e-10


def test_unsupported_combinations_are_rejected():
    mg = _mg()
    with pytest.raises(mg.MGError) as e:
        Problem(65, 64, periodic_y=True, q1="annulus", smoother="gstri_y").solver()
    assert e.value.status == mg.MG_EUNSUPPORTED
    with pytest.raises(mg.MGError) as e:
        mg.BatchedSolver([(65, 65), (33, 33)], [1.0, 0.1], smoother="gsadi")
    assert e.value.status == mg.MG_EUNSUPPORTED
    with pytest.raises(mg.MGError) as e:
        Problem(65, 65, smoother="tri_x", omega=0.0).solver()
    assert e.value.status == mg.MG_EINVAL


@pytest.mark.parametrize("smoother", ["tri_x", "gstri_x"])
def test_long_lines_use_the_thread_per_line_solver(smoother):
    """4609 x 17 nodes: the finest x lines (4607 unknowns, 4 x 4607 FP64 values
    > 140 KB of LDS) are solved by one thread each with the Thomas factors from
    setup, the coarser ones by cyclic reduction; both agree with the oracle.
    A line solve is global along the line, so two correct solve orders differ
    by about cond(T) u: eps = 0.01 keeps cond(T) near 2.5e3 on these lines
    (at eps = 4 it is 6e5 and the difference reaches 1e-12)."""
    p = Problem(4609, 17, eps=0.01, smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(4609, 17, 2), np.zeros((17, 4609)), 3)


@pytest.mark.parametrize("cta", [300, 5000])
@pytest.mark.parametrize("smoother", ["adi", "gsadi"])
def test_coarse_levels_in_global_memory(smoother, cta):
    """Levels of at most `cta` nodes run in the one-workgroup coarse kernel
    reading global memory (one thread per line, Thomas factors from setup);
    the default keeps them in LDS (cyclic reduction over all lines at once)."""
    p = Problem(129, 129, eps=0.05, smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(129, 129, 2), W.uniform_field(129, 129, 1), 3, coarse_cta_nodes=cta)


@pytest.mark.parametrize("case", [
    dict(nx=1025, ny=33, eps=0.05, smoother="gstri_x"),
    dict(nx=1025, ny=33, eps=0.05, smoother="tri_x", omega=0.8),
    dict(nx=33, ny=1025, eps=50.0, smoother="gstri_y"),
    dict(nx=33, ny=1025, eps=50.0, smoother="tri_y", omega=0.8),
], ids=["gstri_x", "tri_x", "gstri_y", "tri_y"])
def test_long_lines_by_cyclic_reduction(case):
    """Lines of 1023 unknowns (the finest lines of the 1025^2 workload) through
    the launched kernels (x lines: cyclic reduction; y lines of 128 or more
    unknowns: segments and separators, k_line_y): coarse_cta_nodes = 1 keeps
    every level but the coarsest out of the one-workgroup kernel.  Per cycle 1e-12
    against the oracle.  Cyclic reduction's forward error on a line is about
    cond(T) log2(m) u, against cond(T) u for the oracle's sparse LU, so the
    cases keep cond(T) near 1e2: 1025 x 33 with eps = 0.05 (x lines:
    (4 * 0.05 * 1024^2 + 2 * 32^2) / (2 * 32^2) = 103) and 33 x 1025 with
    eps = 50 (y lines: (4 * 1024^2 + 100 * 32^2) / (100 * 32^2) = 42).  At
    eps = 1 the x lines have cond(T) = 2e3 and the difference reaches
    2.7e-12 after one cycle, the size that bound predicts."""
    p = Problem(**case)
    check_parity(p, W.normal_field(p.nx, p.ny, 2), W.uniform_field(p.nx, p.ny, 1), 3, coarse_cta_nodes=1)


@pytest.mark.parametrize("case", [
    dict(nx=45, ny=257, eps=1.0, smoother="gstri_y"),
    dict(nx=45, ny=257, eps=10.0, smoother="tri_y", omega=0.8),
    dict(nx=33, ny=513, eps=10.0, smoother="gsadi"),
    dict(nx=161, ny=129, eps=1.0, smoother="gsadi"),
], ids=["gstri_y-257", "tri_y-257", "gsadi-513", "gsadi-129"])
def test_segmented_y_lines_per_cycle(case):
    """y lines through the segment-and-separator kernel (k_line_y): 43 or 31
    lines (colours of 22/21 and 16/15 lines, so the last workgroup of four
    lines is ragged), lines of 255 and 511 unknowns (4 and 8 nodes per
    segment, 63 separators) and, on 161 x 129, lines of 127 unknowns that
    stay on cyclic reduction beside 159-long x lines.  Per cycle 1e-12
    against the oracle; the y lines keep cond(T) below 1e2."""
    p = Problem(**case)
    check_parity(p, W.normal_field(p.nx, p.ny, 2), W.uniform_field(p.nx, p.ny, 1), 3, coarse_cta_nodes=1)


def test_segmented_y_lines_nine_point_cells():
    """y lines of a 9-point operator with per-cell coefficients on the finest
    level (Gaussian random field, 257^2): the line couplings and the six
    off-line couplings come from the cells, the coarser levels' from the
    Galerkin bands."""
    p = Problem(257, 257, q1="grf", smoother="gstri_y")
    check_parity(p, W.normal_field(257, 257, 4), np.zeros((257, 257)), 2, coarse_cta_nodes=1)
