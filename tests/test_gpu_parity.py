"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  FP64 iterates must agree to 1e-12 relative max-norm
after every cycle; integer outcomes (status, cycle counts) must agree."""

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W
from tests.problems import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARITY = 1e-12  # relative max-norm per cycle, FP64
# Residual norms near convergence are ~1e-10 r0 and are evaluated as b - A x
# with terms of size ||A|| |x|; their FP64 rounding floor (eps_mach ||A|| |x|
# per entry) is below 1e-13 r0 on these grids, so histories are compared with
# that absolute slack on top of a relative 1e-8.
HIST_ATOL = 1e-13


def _mg():
    from paper_0805_3041_amd import mg
    return mg


def gpu_iterates(solver, rhs, x0, k):
    """x_1..x_k by resuming one cycle at a time (the cycle is stationary)."""
    r = torch.tensor(rhs, device="cuda")
    x = torch.tensor(x0, device="cuda")
    out = []
    for _ in range(k):
        info = solver.solve(r, x, tol=1e-300, max_cycles=1, history=False)
        assert info.status in (0, 1)
        out.append(x.cpu().numpy().copy())
    return out


def oracle_iterates(h, g, rhs, x0, k):
    b = g.pack(rhs)
    x = g.pack(x0)
    out = []
    for _ in range(k):
        x = O.mg_cycle(h, 0, x, b, h.opts.cycle)
        out.append(x.copy())
    return out


def dirichlet_mask(nx, ny, periodic_y=False):
    """Stored nodes that are Dirichlet boundary nodes: columns 0 and nx - 1,
    and rows 0 and ny - 1 unless y is periodic."""
    m = np.zeros((ny, nx), dtype=bool)
    m[:, 0] = m[:, -1] = True
    if not periodic_y:
        m[0, :] = m[-1, :] = True
    return m


def check_parity(p: Problem, rhs, x0, k, coarse_cta_nodes=0, **extra):
    g = p.grid()
    h = p.oracle()
    s = p.solver(coarse_cta_nodes=coarse_cta_nodes, **extra)
    x0 = np.array(x0, dtype=np.float64)
    bnd = dirichlet_mask(p.nx, p.ny, p.periodic_y)
    if bnd.any():
        x0[bnd] = 7.0  # the solve must overwrite the boundary with zeros
    try:
        xs_g = gpu_iterates(s, rhs, x0, k)
    finally:
        s.close()
    xs_o = oracle_iterates(h, g, rhs, g.unpack(g.pack(x0)), k)
    worst = 0.0
    for c, (xg, xo) in enumerate(zip(xs_g, xs_o), 1):
        # mg_solve writes zero at every Dirichlet boundary node
        assert np.all(xg[bnd] == 0.0), f"cycle {c}: nonzero Dirichlet boundary value"
        err = np.abs(g.pack(xg) - xo).max() / np.abs(xo).max()
        worst = max(worst, err)
        assert err <= PARITY, f"cycle {c}: relative max-norm difference {err:.3e}"
    return worst


# ----------------------------------------------------------------------------- poisson65 (Jacobi)


@pytest.mark.parametrize("cta", [0, 1])
@pytest.mark.parametrize("rhs_kind", ["manufactured", "normal"])
def test_poisson65_jacobi_per_cycle(cta, rhs_kind):
    p = Problem(65, 65, smoother="jacobi", omega=0.8)
    rhs = W.manufactured_sine(65)[0] if rhs_kind == "manufactured" else W.normal_field(65, 65, 0)
    check_parity(p, rhs, np.zeros((65, 65)), 9, coarse_cta_nodes=cta)


def test_poisson65_solve_status_cycles_and_error():
    p = Problem(65, 65, smoother="jacobi", omega=0.8)
    f, u = W.manufactured_sine(65)
    g = p.grid()
    ref = O.solve(p.oracle(), g.pack(f), np.zeros(g.n_unknowns), 1e-10, 100)
    s = p.solver()
    x = torch.zeros((65, 65), dtype=torch.float64, device="cuda")
    info = s.solve(torch.tensor(f, device="cuda"), x, 1e-10, 100)
    s.close()
    assert info.status == 0 and info.cycles == ref.cycles
    np.testing.assert_allclose(info.history, ref.history, rtol=1e-8, atol=HIST_ATOL * ref.history[0])
    xh = np.pi / 128
    err = np.abs(x.cpu().numpy() - u).max()
    assert abs(err - ((xh / np.sin(xh)) ** 2 - 1)) < 1e-8


# ----------------------------------------------------------------------------- anisotropic, red-black GS


@pytest.mark.parametrize("eps", W.ANISO_EPS)
@pytest.mark.parametrize("x0", ["zero", "uniform"])
def test_aniso_rbgs_per_cycle(eps, x0):
    n = 129
    p = Problem(n, n, eps=eps, smoother="rbgs")
    check_parity(p, W.aniso_rhs(n, 2), W.aniso_x0(n, x0, 1), 3, coarse_cta_nodes=300)


@pytest.mark.parametrize("nu", [1, 2, 3, 4])
def test_aniso_rbgs_smoothing_steps(nu):
    n = 257
    p = Problem(n, n, eps=0.1, smoother="rbgs", nu_pre=nu, nu_post=nu)
    check_parity(p, W.aniso_rhs(n, 2), W.aniso_x0(n, "uniform", 1), 2)


@pytest.mark.parametrize("cta", [1, 300, 5000, 100000])
def test_cta_threshold_is_bitwise_invisible(cta):
    """Where the coarse levels run (per-op launches or the single-workgroup kernel)
    does not change a single bit of the iterate."""
    n = 129
    p = Problem(n, n, eps=0.01, smoother="rbgs")
    rhs = W.aniso_rhs(n, 2)
    ref = p.solver(coarse_cta_nodes=1)
    got = p.solver(coarse_cta_nodes=cta)
    try:
        a = gpu_iterates(ref, rhs, np.zeros((n, n)), 2)
        b = gpu_iterates(got, rhs, np.zeros((n, n)), 2)
    finally:
        ref.close()
        got.close()
    for xa, xb in zip(a, b):
        assert np.array_equal(xa, xb)


def test_ragged_rectangular_grid():
    """97 x 49 nodes (3 * 2^5 + 1 by 3 * 2^4 + 1): coarsest 7 x 4, 10 unknowns."""
    p = Problem(97, 49, eps=0.3, smoother="rbgs")
    g = p.grid()
    assert O.hierarchy_grids(g)[-1].nx == 7
    check_parity(p, W.normal_field(97, 49, 5), np.zeros((49, 97)), 3, coarse_cta_nodes=400)


def test_periodic_5pt():
    p = Problem(65, 64, periodic_y=True, eps=0.5, smoother="rbgs")
    check_parity(p, W.normal_field(65, 64, 6, True), np.zeros((64, 65)), 3, coarse_cta_nodes=600)


@pytest.mark.parametrize("smoother", ["jacobi", "rbgs", "gs4c"])
def test_v_cycle(smoother):
    p = Problem(65, 65, eps=1.0, smoother=smoother, cycle="V", nu_pre=1, nu_post=2)
    check_parity(p, W.normal_field(65, 65, 7), np.zeros((65, 65)), 3, coarse_cta_nodes=300)


@pytest.mark.parametrize("cta", [0, 300])
@pytest.mark.parametrize("smoother", ["jacobi", "rbgs", "gstri_y"])
def test_w_cycle(smoother, cta):
    """W-cycles (two recursive W-cycles per level) through the fused passes,
    the one-workgroup coarse kernel in LDS (cta 0) or in global memory
    (cta 300), and the line sweeps."""
    p = Problem(129, 129, eps=0.1, smoother=smoother, cycle="W", nu_pre=1, nu_post=1)
    check_parity(p, W.normal_field(129, 129, 7), W.uniform_field(129, 129, 1), 3, coarse_cta_nodes=cta)


def test_w_cycle_annulus():
    p = Problem(129, 128, periodic_y=True, q1="annulus", smoother="gs4c", cycle="W")
    check_parity(p, W.normal_field(129, 128, 3, True), np.zeros((128, 129)), 2)


@pytest.mark.slow
def test_aniso1025_full_size_two_cycles():
    n = 1025
    p = Problem(n, n, eps=1e-2, smoother="rbgs")
    check_parity(p, W.aniso_rhs(n, 2), W.aniso_x0(n, "uniform", 1), 2)


# ----------------------------------------------------------------------------- 9-point Q1


@pytest.mark.parametrize("n", [33, 65, 129])
def test_annulus_gs4c_per_cycle(n):
    p = Problem(n, n - 1, periodic_y=True, q1="annulus", smoother="gs4c")
    check_parity(p, W.annulus_rhs(n, n - 1, 3), np.zeros((n - 1, n)), 3, coarse_cta_nodes=300)


@pytest.mark.parametrize("smoother", ["gs4c", "jacobi"])
def test_grf_q1_per_cycle(smoother):
    n = 65
    p = Problem(n, n, q1="grf", smoother=smoother, omega=0.8)
    f, _ = W.manufactured_sine(n)
    check_parity(p, f, np.zeros((n, n)), 3, coarse_cta_nodes=300)


def test_grf_q1_galerkin_levels_all_on_gpu():
    """129^2 with per-op launches on every level (Galerkin 2-D bands on each)."""
    n = 129
    p = Problem(n, n, q1="grf", smoother="gs4c")
    check_parity(p, W.normal_field(n, n, 8), np.zeros((n, n)), 2, coarse_cta_nodes=1)


# ----------------------------------------------------------------------------- solve-level behaviour


def test_residual_matches_oracle():
    n = 129
    p = Problem(n, n, eps=0.2)
    g = p.grid()
    rhs = W.normal_field(n, n, 9)
    x = W.uniform_field(n, n, 10)
    x_dirty = x.copy()
    x_dirty[0, :] = 5.0  # boundary values are not unknowns and must be ignored
    s = p.solver()
    r = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    nrm = s.residual(torch.tensor(rhs, device="cuda"), torch.tensor(x_dirty, device="cuda"), r)
    s.close()
    ro = g.pack(rhs) - p.oracle().A[0] @ g.pack(x)
    assert abs(nrm - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(ro)
    np.testing.assert_allclose(g.pack(r.cpu().numpy()), ro, atol=1e-12 * np.abs(ro).max())
    assert np.all(r.cpu().numpy()[0, :] == 0)


def test_diverging_jacobi_reports_diverged():
    n = 33
    p = Problem(n, n, smoother="jacobi", omega=2.5)
    g = p.grid()
    rhs = W.normal_field(n, n, 11)
    ref = O.solve(p.oracle(), g.pack(rhs), np.zeros(g.n_unknowns), 1e-10, 200)
    s = p.solver()
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = s.solve(torch.tensor(rhs, device="cuda"), x, 1e-10, 200)
    s.close()
    assert ref.status == O.DIVERGED
    assert info.status == _mg().MG_DIVERGED and info.cycles == ref.cycles


def test_max_cycles_reports_not_converged():
    n = 65
    p = Problem(n, n, eps=1e-3)
    s = p.solver()
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = s.solve(torch.tensor(W.normal_field(n, n, 12), device="cuda"), x, 1e-10, 1)
    s.close()
    assert info.status == _mg().MG_NOT_CONVERGED and info.cycles == 1


def test_zero_rhs_returns_immediately():
    n = 65
    s = Problem(n, n).solver()
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = s.solve(torch.zeros((n, n), dtype=torch.float64, device="cuda"), x, 1e-10, 10)
    s.close()
    assert info.status == 0 and info.cycles == 0 and torch.all(x == 0)


def test_resume_is_bitwise_equal():
    n = 129
    p = Problem(n, n, eps=0.05)
    rhs = torch.tensor(W.normal_field(n, n, 13), device="cuda")
    s = p.solver()
    a = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    s.solve(rhs, a, 1e-300, 5, history=False)
    b = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    s.solve(rhs, b, 1e-300, 2, history=False)
    s.solve(rhs, b, 1e-300, 3, history=False)
    s.close()
    assert torch.equal(a, b)


@pytest.mark.parametrize("eps", [1.0, 0.1, 0.01])
def test_fp64_cycles_to_tolerance_match_oracle(eps):
    n = 129
    p = Problem(n, n, eps=eps)
    g = p.grid()
    rhs = W.aniso_rhs(n, 2)
    ref = O.solve(p.oracle(), g.pack(rhs), np.zeros(g.n_unknowns), 1e-10, 2000)
    s = p.solver()
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = s.solve(torch.tensor(rhs, device="cuda"), x, 1e-10, 2000)
    s.close()
    assert info.status == 0 and info.cycles == ref.cycles, (info.cycles, ref.cycles)
    m = min(len(ref.history), len(info.history))
    np.testing.assert_allclose(info.history[:m], ref.history[:m], rtol=1e-8, atol=HIST_ATOL * ref.history[0])
    assert np.abs(g.pack(x.cpu().numpy()) - ref.x).max() <= 1e-9 * np.abs(ref.x).max()


# ----------------------------------------------------------------------------- mixed precision


@pytest.mark.parametrize("eps", [1.0, 0.1])
def test_mixed_precision_reaches_tolerance(eps):
    """Mixed form: the oracle's FP64 residual of the GPU solution is <= tol * r0
    (plus FP64 evaluation noise), and it needs at most 2 more cycles than FP64."""
    n = 257
    p = Problem(n, n, eps=eps)
    g = p.grid()
    h = p.oracle()
    rhs = W.aniso_rhs(n, 2)
    ref = O.solve(h, g.pack(rhs), np.zeros(g.n_unknowns), 1e-10, 500)
    s = p.solver(precision="mixed")
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = s.solve(torch.tensor(rhs, device="cuda"), x, 1e-10, 500)
    s.close()
    assert info.status == 0
    assert info.cycles <= ref.cycles + 2
    r = O.residual_norm(h, g.pack(rhs), g.pack(x.cpu().numpy()))
    assert r <= 1.05e-10 * ref.history[0]
    diff = np.abs(g.pack(x.cpu().numpy()) - ref.x).max() / np.abs(ref.x).max()
    assert diff < 1e-7, diff


def test_mixed_first_cycle_close_to_oracle_mixed():
    """One mixed outer step against the oracle's mixed step (FP32 inner cycle):
    equal up to FP32 rounding of the correction."""
    n = 129
    p = Problem(n, n, eps=0.3)
    g = p.grid()
    h = p.oracle()
    rhs = W.aniso_rhs(n, 2)
    ref = O.solve_mixed(h, g.pack(rhs), np.zeros(g.n_unknowns), 1e-300, 2)
    s = p.solver(precision="mixed")
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    s.solve(torch.tensor(rhs, device="cuda"), x, 1e-300, 2, history=False)
    s.close()
    diff = np.abs(g.pack(x.cpu().numpy()) - ref.x).max() / np.abs(ref.x).max()
    assert diff < 1e-5, diff


# ----------------------------------------------------------------------------- fused tiles


FUSED_CASES = [
    dict(p=dict(nx=129, ny=129, eps=0.01, smoother="rbgs"), cta=300),
    dict(p=dict(nx=257, ny=257, eps=0.1, smoother="rbgs", nu_pre=1, nu_post=3), cta=300),
    dict(p=dict(nx=257, ny=257, eps=1.0, smoother="rbgs", nu_pre=4, nu_post=4), cta=300),
    dict(p=dict(nx=65, ny=64, periodic_y=True, eps=0.5, smoother="rbgs"), cta=100),
    dict(p=dict(nx=97, ny=49, eps=0.3, smoother="rbgs"), cta=100),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c"), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c"), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="jacobi", nu_pre=3, nu_post=1), cta=300),
    dict(p=dict(nx=65, ny=65, smoother="jacobi"), cta=1),
    dict(p=dict(nx=129, ny=129, eps=0.2, smoother="rbgs", cycle="V"), cta=100, tile=(16, 4)),
    dict(p=dict(nx=129, ny=129, eps=0.2, smoother="gs4c"), cta=100, tile=(128, 32)),
    dict(p=dict(nx=257, ny=257, eps=0.05, smoother="rbgs"), cta=100, tile=(32, 8)),
    dict(p=dict(nx=289, ny=161, eps=0.3, smoother="rbgs"), cta=100, wide_ty=6),
    dict(p=dict(nx=257, ny=256, periodic_y=True, q1="annulus", smoother="gs4c"), cta=300, wide_ty=10),
    dict(p=dict(nx=257, ny=256, periodic_y=True, q1="annulus", smoother="jacobi", nu_pre=2, nu_post=3), cta=300),
    dict(p=dict(nx=257, ny=257, eps=0.1, smoother="rbgs", sor=1.4), cta=300),
    dict(p=dict(nx=257, ny=257, q1="sphere", smoother="gs4c"), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c", sor=0.8), cta=300),
    dict(p=dict(nx=257, ny=256, periodic_y=True, q1="annulus", smoother="gs4c", sor=1.25), cta=300, wide_ty=10),
]


@pytest.mark.parametrize("mode", ["narrow", "wide"])
@pytest.mark.parametrize("case", FUSED_CASES, ids=[str(i) for i in range(len(FUSED_CASES))])
def test_fused_tiles_equal_per_op_bitwise(case, mode):
    """The LDS-tiled passes (small tiles, and 128-column wide tiles forced on
    every fused level) give the per-op kernels' iterate bit for bit, and both
    match the oracle."""
    p = Problem(**case["p"])
    rhs = W.normal_field(p.nx, p.ny, 21, p.periodic_y)
    x0 = W.uniform_field(p.nx, p.ny, 22, p.periodic_y)
    tx, ty = case.get("tile", (0, 0))
    if mode == "wide":
        if tx:
            pytest.skip("explicit small-tile width")
        ty = case.get("wide_ty", 0)
    a = p.solver(coarse_cta_nodes=case["cta"], tile_mode="per_op")
    b = p.solver(coarse_cta_nodes=case["cta"], tile_mode=mode, tile_x=tx, tile_y=ty)
    try:
        xa = gpu_iterates(a, rhs, x0, 2)
        xb = gpu_iterates(b, rhs, x0, 2)
    finally:
        a.close()
        b.close()
    for u, v in zip(xa, xb):
        assert np.array_equal(u, v)
    g = p.grid()
    xo = oracle_iterates(p.oracle(), g, rhs, x0, 2)
    for u, v in zip(xb, xo):
        assert np.abs(g.pack(u) - v).max() <= PARITY * np.abs(v).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_solve_matches_per_op_solve(precision):
    """Whole solves (stopping test fused into the finest post-pass) agree with the per-op path."""
    n = 257
    p = Problem(n, n, eps=0.05)
    rhs = torch.tensor(W.aniso_rhs(n, 2), device="cuda")
    out = []
    for mode in ("per_op", "fused", "wide"):
        s = p.solver(precision=precision, tile_mode=mode)
        x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        info = s.solve(rhs, x, 1e-10, 1000)
        s.close()
        out.append((info, x.cpu().numpy()))
    (ia, xa) = out[0]
    for ib, xb in out[1:]:
        assert ia.status == ib.status == 0 and ia.cycles == ib.cycles
        assert np.array_equal(xa, xb)
        # same iterates; the norms are summed in a different order (tiles vs rows)
        np.testing.assert_allclose(ia.history, ib.history, rtol=1e-14, atol=0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_tile_per_cu_on_the_finest_level(precision):
    """1025^2 nodes: between one and two wide tiles per CU the tile chooser
    takes tiles tall enough for at most one per CU (256 workgroups); two
    cycles give the per-op kernels' iterate bit for bit."""
    n = 1025
    p = Problem(n, n, eps=0.01)
    rhs = torch.tensor(W.aniso_rhs(n, 2), device="cuda")
    x0 = torch.tensor(W.uniform_field(n, n, 22), device="cuda")
    out = []
    for mode in ("per_op", "fused"):
        s = p.solver(precision=precision, tile_mode=mode, tune="off")
        try:
            if mode == "fused":
                for which in (0, 1):
                    info = s.pass_info(0, which)
                    assert info["wide"] == 1 and info["workgroups"] <= 256, info
            x = x0.clone()
            s.solve(rhs, x, 1e-300, 2, history=False)
            out.append(x)
        finally:
            s.close()
    assert torch.equal(out[0], out[1])


# ----------------------------------------------------------------------------- SOR


SOR_CASES = [
    dict(p=dict(nx=65, ny=65, eps=0.1, smoother="rbgs", sor=1.3), cta=0),      # all in the LDS interpreter
    dict(p=dict(nx=129, ny=129, eps=0.1, smoother="rbgs", sor=1.3), cta=300),  # fused levels + interpreter
    dict(p=dict(nx=129, ny=129, eps=0.1, smoother="rbgs", sor=0.7), cta=5000),  # interpreter on global memory
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c", sor=1.2), cta=300),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c", sor=1.2), cta=300),
]


@pytest.mark.parametrize("case", SOR_CASES, ids=[str(i) for i in range(len(SOR_CASES))])
def test_sor_per_cycle(case):
    """Over- and under-relaxed colour Gauss-Seidel (SOR, C = D + omega L)
    against the oracle, cycle by cycle."""
    p = Problem(**case["p"])
    check_parity(p, W.normal_field(p.nx, p.ny, 2, p.periodic_y), W.uniform_field(p.nx, p.ny, 1, p.periodic_y), 3,
                 coarse_cta_nodes=case["cta"])


def test_sor_mixed_precision_reaches_tolerance():
    from oracle import mg_oracle as O
    n = 257
    p = Problem(n, n, eps=0.05, sor=1.2)
    g = p.grid()
    rhs = W.normal_field(n, n, 2)
    s = p.solver(precision="mixed")
    try:
        x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        info = s.solve(torch.tensor(rhs, device="cuda"), x, tol=1e-10, max_cycles=200)
    finally:
        s.close()
    assert info.status == 0
    h = p.oracle()
    b = g.pack(rhs)
    rel = O.residual_norm(h, b, g.pack(x.cpu().numpy())) / O.residual_norm(h, b, np.zeros_like(b))
    assert rel <= 1e-10


def test_sor_zero_stands_for_one():
    """sor = 0 (a zero-initialised option struct) is sor = 1, plain
    Gauss-Seidel, bit for bit; another factor changes the iterate."""
    n = 129
    rhs = torch.tensor(W.normal_field(n, n, 2), device="cuda")
    out = []
    for sor in (1.0, 0.0, 1.3):
        s = Problem(n, n, eps=0.1, sor=sor).solver(coarse_cta_nodes=300)
        try:
            x = torch.zeros_like(rhs)
            s.solve(rhs, x, 1e-300, 3, history=False)
            out.append(x)
        finally:
            s.close()
    assert torch.equal(out[0], out[1]) and not torch.equal(out[0], out[2])


# ----------------------------------------------------------------------------- asymptotic rate

RATE_CASES = [
    dict(nx=33, ny=33, eps=1.0, smoother="rbgs"),
    dict(nx=33, ny=33, eps=0.1, smoother="rbgs"),
    dict(nx=33, ny=32, periodic_y=True, q1="annulus", smoother="gs4c"),
    dict(nx=17, ny=17, eps=1.0, smoother="jacobi"),
]


@pytest.mark.parametrize("case", RATE_CASES, ids=[str(i) for i in range(len(RATE_CASES))])
def test_asymptotic_rate_matches_cycle_matrix_spectral_radius(case):
    """With b = 0 the GPU's F-cycles are a power iteration of the cycle's
    iteration matrix M (built by the oracle from unit vectors): the measured
    asymptotic rate (geometric mean of the residual ratios over the last 10
    of 40 cycles, random start) is within 5 % of the spectral radius of M."""
    p = Problem(**case)
    M = O.cycle_matrix(p.oracle(), "F")
    rho = max(abs(np.linalg.eigvals(M)))
    s = p.solver()
    x = torch.tensor(W.uniform_field(p.nx, p.ny, 7, p.periodic_y), device="cuda")
    rhs = torch.zeros_like(x)
    info = s.solve(rhs, x, tol=1e-300, max_cycles=40, history=True)
    s.close()
    h = np.asarray(info.history)
    assert len(h) == 41 and np.all(h > 0)
    rate = (h[-1] / h[-11]) ** 0.1
    assert abs(rate - rho) <= 0.05 * rho, (rate, rho)


# ----------------------------------------------------------------------------- nested-iteration start vector


NESTED_CASES = [
    dict(nx=65, ny=65, eps=1.0, smoother="rbgs", cycle="F"),
    dict(nx=129, ny=129, eps=0.1, smoother="rbgs", cycle="V"),
    dict(nx=65, ny=65, eps=1.0, smoother="jacobi", cycle="W"),
    dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c", cycle="F"),
    dict(nx=129, ny=129, eps=1e-3, smoother="gstri_y", cycle="F"),
]


@pytest.mark.parametrize("case", NESTED_CASES, ids=[str(i) for i in range(len(NESTED_CASES))])
def test_nested_start_matches_oracle(case):
    """mg_start_nested against the oracle's nested iteration (1e-12), then a
    solve from it needs no more cycles than from zero."""
    p = Problem(**case)
    g = p.grid()
    rhs = p.rhs(5)
    want = O.nested_start(p.oracle(), g.pack(rhs))
    s = p.solver()
    try:
        r = torch.tensor(rhs, device="cuda")
        x = torch.full_like(r, 3.0)  # overwritten
        s.nested_start(r, x)
        got = x.cpu().numpy()
        err = np.abs(g.pack(got) - want).max() / np.abs(want).max()
        assert err <= PARITY, err
        assert np.all(got[dirichlet_mask(p.nx, p.ny, p.periodic_y)] == 0.0)
        info_n = s.solve(r, x, tol=1e-10, max_cycles=200)
        x.zero_()
        info_z = s.solve(r, x, tol=1e-10, max_cycles=200)
    finally:
        s.close()
    assert info_n.status == 0 and info_z.status == 0
    assert info_n.cycles <= info_z.cycles


def test_nested_start_mixed_precision():
    """The mixed form runs the nested iteration in FP32: the start is within
    FP32 rounding of the oracle's FP64 one and the solve converges from it."""
    p = Problem(257, 257, eps=1.0, smoother="rbgs")
    g = p.grid()
    rhs = p.rhs(5)
    want = O.nested_start(p.oracle(), g.pack(rhs))
    s = p.solver(precision="mixed")
    try:
        r = torch.tensor(rhs, device="cuda")
        x = torch.zeros_like(r)
        s.nested_start(r, x)
        err = np.abs(g.pack(x.cpu().numpy()) - want).max() / np.abs(want).max()
        assert err <= 1e-5, err
        info = s.solve(r, x, tol=1e-10, max_cycles=100)
    finally:
        s.close()
    assert info.status == 0


@pytest.mark.parametrize("levels", [2, 3, 4, 5])
def test_level_count(levels):
    """Fewer levels (the "Grid levels" study): the coarsest grid grows (up to
    33^2 = 961 unknowns for two levels) and is still solved exactly."""
    p = Problem(65, 65, eps=0.3, smoother="rbgs", levels=levels)
    check_parity(p, W.normal_field(65, 65, 2), W.uniform_field(65, 65, 1), 3)


# ----------------------------------------------------------------------------- options of the boundary


def test_mixed_inner_cycles_match_oracle():
    """inner_cycles = 2: each outer step gives the FP32 correction two cycles
    from zero before x += e.  The first step agrees with the oracle's mixed
    form to FP32 rounding: each of the two FP32 cycles adds rounding of the
    size the single-cycle bound (1e-5) allows, so the bound here is 2e-5; the
    solve reaches 1e-10 by the oracle's FP64 residual in fewer outer steps
    than with one inner cycle."""
    n = 129
    p = Problem(n, n, eps=0.1)
    g = p.grid()
    h = p.oracle()
    rhs = W.aniso_rhs(n, 2)
    b = g.pack(rhs)
    one = O.solve_mixed(h, b, np.zeros(g.n_unknowns), 1e-300, 1, inner=2)
    s = p.solver(precision="mixed", inner_cycles=2)
    try:
        r = torch.tensor(rhs, device="cuda")
        x = torch.zeros_like(r)
        s.solve(r, x, 1e-300, 1, history=False)
        err = np.abs(g.pack(x.cpu().numpy()) - one.x).max() / np.abs(one.x).max()
        assert err <= 2e-5, err
        x.zero_()
        info2 = s.solve(r, x, 1e-10, 200)
        xs = x.cpu().numpy()
    finally:
        s.close()
    s1 = p.solver(precision="mixed")
    try:
        x1 = torch.zeros_like(r)
        info1 = s1.solve(r, x1, 1e-10, 200)
    finally:
        s1.close()
    assert info2.status == 0 and info1.status == 0
    assert O.residual_norm(h, b, g.pack(xs)) <= 1.0001e-10 * np.linalg.norm(b)
    assert info2.cycles < info1.cycles, (info2.cycles, info1.cycles)
    ref = O.solve_mixed(h, b, np.zeros(g.n_unknowns), 1e-10, 200, inner=2)
    assert abs(info2.cycles - ref.cycles) <= 1, (info2.cycles, ref.cycles)


@pytest.mark.parametrize("case", [
    dict(nx=65, ny=65, eps=1.0, smoother="gs4c"),
    dict(nx=129, ny=129, eps=0.1, smoother="gs4c", cycle="V"),
    dict(nx=97, ny=49, eps=0.3, smoother="jacobi", omega=0.8),
    dict(nx=129, ny=128, periodic_y=True, eps=1.0, smoother="gs4c"),
], ids=["65-gs4c", "129-V", "97x49-jacobi", "periodic"])
@pytest.mark.parametrize("cta", [0, 1])
def test_galerkin_coarse_levels_of_5point_problems(case, cta):
    """coarse_op = galerkin on a 5-point problem: coarse operators R A P
    (9-point) through the band kernels, per cycle against the oracle's
    Galerkin hierarchy (1e-12), fused passes and the coarse-level kernel."""
    p = Problem(coarse_op="galerkin", **case)
    check_parity(p, W.normal_field(p.nx, p.ny, 3, p.periodic_y), np.zeros((p.ny, p.nx)), 3,
                 coarse_cta_nodes=300 if cta else 0)


ROW_HALO_CASES = [
    # (problem, nu_pre/nu_post): four colours take a row halo of half their
    # colour steps (+ 2 rows for the pre-pass's defect and restriction)
    dict(p=dict(nx=129, ny=129, eps=0.3, smoother="gs4c")),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c")),
    dict(p=dict(nx=129, ny=129, eps=1.0, smoother="gs4c", nu_pre=1, nu_post=3)),
    dict(p=dict(nx=97, ny=97, q1="grf", smoother="gs4c", sor=1.2)),
]


@pytest.mark.parametrize("ty", [2, 4, 6, 10, 16])
@pytest.mark.parametrize("case", ROW_HALO_CASES, ids=[str(i) for i in range(len(ROW_HALO_CASES))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_four_colour_row_halo_is_bitwise_invisible(case, ty, precision):
    """Wide tiles with four colours sweep TY + 2 Hy rows, Hy about half the
    column halo: from tiles of two output rows (every row of the region in
    the halo) to sixteen, two cycles give the per-op kernels' iterates bit
    for bit (the mixed form's FP32 cycles included)."""
    p = Problem(**case["p"])
    rhs = W.normal_field(p.nx, p.ny, 61, p.periodic_y)
    x0 = W.uniform_field(p.nx, p.ny, 62, p.periodic_y)
    a = p.solver(precision=precision, coarse_cta_nodes=300, tile_mode="per_op")
    b = p.solver(precision=precision, coarse_cta_nodes=300, tile_mode="wide", tile_y=ty)
    try:
        info = b.pass_info(0, 0)
        nu = p.nu_pre
        assert info["wide"] == 1 and info["halo"] == 4 * nu + 2 and info["halo_y"] == 2 * nu + 2, info
        xa = gpu_iterates(a, rhs, x0, 2)
        xb = gpu_iterates(b, rhs, x0, 2)
    finally:
        a.close()
        b.close()
    for u, v in zip(xa, xb):
        assert np.array_equal(u, v)
