"""Mixed form with the residual formed inside the finest pre-pass.

When the first finest pre-pass of an outer step runs on wide tiles from a
zero correction, it forms r = b - A x of the FP64 level itself (the same
products as the residual kernel, so r is the same to the bit) and the
stopping test of a cycle's result is taken at the start of the next cycle,
or by a check of its own after the last queued cycle.  These tests compare
that path with the residual kernel's path, which a pre-pass tile too tall
for the in-pass residual (more than 96 region rows) keeps: iterates equal
bit for bit, same statuses and cycle counts, residual histories equal up to
the order of the norm's sums (tiles against column strips)."""

import numpy as np
import pytest

import workloads as W
from tests.problems import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RESID_ROWS_MAX = 96  # region rows (TY + 2 Hy) the in-pass residual holds per tile

CASES = [
    # 9-point, bands constant along y (the annulus operator), four colours
    dict(p=dict(nx=257, ny=256, periodic_y=True, q1="annulus", smoother="gs4c"), fit=16),
    # 5-point, red-black
    dict(p=dict(nx=257, ny=257, eps=0.05, smoother="rbgs"), fit=24),
    # 5-point, damped Jacobi (a third LDS array per row), non-square
    dict(p=dict(nx=193, ny=129, eps=0.5, smoother="jacobi", omega=0.8), fit=20),
]


def _mg():
    from paper_0805_3041_amd import mg
    return mg


def _pair(p, fit):
    """Two mixed solvers on wide tiles: one whose finest pre-pass forms the
    residual, one whose pre-pass tile is too tall for it."""
    a = p.solver(precision="mixed", tile_mode="wide", tile_y=fit)
    ia = a.pass_info(0, 0)
    tall = RESID_ROWS_MAX + 2 - 2 * ia["halo_y"]
    b = p.solver(precision="mixed", tile_mode="wide", tile_y=tall)
    ib = b.pass_info(0, 0)
    assert ia["wide"] == 1 and ia["ty"] + 2 * ia["halo_y"] <= RESID_ROWS_MAX and ia["forms_residual"] == 1, ia
    assert ib["wide"] == 1 and ib["ty"] + 2 * ib["halo_y"] > RESID_ROWS_MAX and ib["forms_residual"] == 0, ib
    return a, b


def _solve(s, rhs, x0, tol, max_cycles):
    x = x0.clone()
    info = s.solve(rhs, x, tol, max_cycles)
    return info, x.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_in_pass_residual_equals_residual_kernel(case):
    mg = _mg()
    p = Problem(**case["p"])
    rhs = torch.tensor(p.rhs(31), device="cuda")
    x0 = torch.tensor(W.uniform_field(p.nx, p.ny, 32, p.periodic_y), device="cuda")
    a, b = _pair(p, case["fit"])
    try:
        for tol, cap in ((1e-10, 200), (1e-300, 3), (1e-300, 1)):
            ia, xa = _solve(a, rhs, x0, tol, cap)
            ib, xb = _solve(b, rhs, x0, tol, cap)
            assert ia.status == ib.status and ia.cycles == ib.cycles, (tol, cap, ia, ib)
            if tol == 1e-10:
                assert ia.status == mg.MG_OK and ia.rel_res <= 1e-10
            else:
                assert ia.status == mg.MG_NOT_CONVERGED and ia.cycles == cap
            assert np.array_equal(xa, xb), (tol, cap)
            assert len(ia.history) == ia.cycles + 1
            np.testing.assert_allclose(ia.history, ib.history, rtol=1e-13, atol=0)
            # a second solve on the same handle starts its state afresh
            ia2, xa2 = _solve(a, rhs, x0, tol, cap)
            assert ia2.cycles == ia.cycles and np.array_equal(xa2, xa)
            np.testing.assert_array_equal(ia2.history, ia.history)
    finally:
        a.close()
        b.close()


def test_in_pass_residual_history_is_the_true_residual():
    """Each recorded norm is ||b - A x_k|| of that cycle's iterate: two capped
    solves of k and k + 1 cycles end on iterates whose oracle residual norms
    are the last two entries of the longer history."""
    p = Problem(257, 256, periodic_y=True, q1="annulus", smoother="gs4c")
    rhs_np = p.rhs(41)
    rhs = torch.tensor(rhs_np, device="cuda")
    x0 = torch.zeros_like(rhs)
    a, b = _pair(p, 16)
    b.close()
    g = p.grid()
    h = p.oracle()
    try:
        i3, x3 = _solve(a, rhs, x0, 1e-300, 3)
        i4, x4 = _solve(a, rhs, x0, 1e-300, 4)
    finally:
        a.close()
    A = h.A[0]
    for x, want in ((x3, i4.history[3]), (x4, i4.history[4])):
        r = g.pack(rhs_np) - A @ g.pack(x)
        assert abs(np.linalg.norm(r) - want) <= 1e-12 * i4.history[0], (np.linalg.norm(r), want)
    np.testing.assert_allclose(i3.history, i4.history[:4], rtol=0, atol=0)


def test_batched_slots_form_their_residual():
    """A batched handle whose same-shape problems share one group (one launch
    per pass, a problem per slot): each problem's iterate equals its own
    single solve bit for bit, with statuses and cycle counts, while problems
    stop at different cycles."""
    mg = _mg()
    n = 257
    eps = [1.0, 0.05, 0.3]
    rhs = [torch.tensor(W.normal_field(n, n, 700 + k), device="cuda") for k in range(len(eps))]
    B = mg.BatchedSolver([(n, n)] * len(eps), eps, smoother="rbgs", precision="mixed", tile_mode="wide", tile_y=24)
    try:
        assert B.schedule()["standalone"] == 1  # one group, a slot per problem
        xb = [torch.zeros_like(r) for r in rhs]
        _, infos = B.solve(rhs, xb, 1e-10, 300)
    finally:
        B.close()
    cycles = set()
    for k, e in enumerate(eps):
        s = mg.Solver(n, n, eps_x=e, smoother="rbgs", precision="mixed", tile_mode="wide", tile_y=24)
        try:
            assert s.pass_info(0, 0)["forms_residual"] == 1
            x = torch.zeros_like(rhs[k])
            info = s.solve(rhs[k], x, 1e-10, 300, history=False)
        finally:
            s.close()
        assert info.status == infos[k].status == mg.MG_OK
        assert info.cycles == infos[k].cycles
        cycles.add(info.cycles)
        assert torch.equal(x, xb[k]), k
    assert len(cycles) > 1


def test_in_pass_residual_with_three_inner_cycles():
    """Three FP32 cycles per outer step (the first pre-pass of a step forms
    the residual, the two later ones read e): iterates equal the residual
    kernel's path bit for bit, capped and to tolerance."""
    mg = _mg()
    p = Problem(257, 256, periodic_y=True, q1="annulus", smoother="gs4c")
    rhs = torch.tensor(p.rhs(51), device="cuda")
    x0 = torch.zeros_like(rhs)
    a = p.solver(precision="mixed", tile_mode="wide", tile_y=16, inner_cycles=3)
    h = a.pass_info(0, 0)["halo_y"]
    b = p.solver(precision="mixed", tile_mode="wide", tile_y=RESID_ROWS_MAX + 2 - 2 * h, inner_cycles=3)
    try:
        assert a.pass_info(0, 0)["forms_residual"] == 1 and b.pass_info(0, 0)["forms_residual"] == 0
        for tol, cap in ((1e-10, 100), (1e-300, 2)):
            ia, xa = _solve(a, rhs, x0, tol, cap)
            ib, xb = _solve(b, rhs, x0, tol, cap)
            assert ia.status == ib.status and ia.cycles == ib.cycles, (ia, ib)
            assert ia.status == (mg.MG_OK if tol == 1e-10 else mg.MG_NOT_CONVERGED)
            assert np.array_equal(xa, xb)
            np.testing.assert_allclose(ia.history, ib.history, rtol=1e-13, atol=0)
    finally:
        a.close()
        b.close()
