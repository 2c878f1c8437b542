"""Coefficient update in an existing handle (mg_update_coeffs): a solve after
the update equals, bit for bit, the solve of a handle set up for the new
coefficients directly (the same kernels on the same operators), on a finest
level that keeps cell copies, the mixed hierarchy, line-smoother factors and
a finest level run by the coarse-level interpreter; the reusable
GradientSolver gives MGSolve's gradients step after step; invalid updates are
rejected."""

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mg():
    from paper_0805_3041_amd import mg
    return mg


def _cells(nx, ny, periodic, seed):
    ncy = ny if periodic else ny - 1
    rng = np.random.default_rng(seed)
    return torch.tensor(np.exp(0.7 * rng.standard_normal((ncy, nx - 1))), device="cuda")


UPDATE_CASES = [
    dict(nx=257, ny=257, opts=dict(smoother="gs4c")),
    dict(nx=257, ny=257, opts=dict(smoother="gs4c", precision="mixed")),
    dict(nx=129, ny=128, periodic=True, opts=dict(smoother="gs4c")),
    dict(nx=129, ny=129, opts=dict(smoother="gsadi", omega=0.8)),
    dict(nx=97, ny=65, opts=dict(smoother="jacobi", omega=0.8, tile_mode="per_op")),
    dict(nx=33, ny=33, opts=dict(smoother="gs4c")),
]


@pytest.mark.parametrize("case", UPDATE_CASES, ids=[str(i) for i in range(len(UPDATE_CASES))])
def test_update_equals_fresh_setup(case):
    mg = _mg()
    nx, ny, per = case["nx"], case["ny"], case.get("periodic", False)
    a1 = _cells(nx, ny, per, 1)
    a2 = _cells(nx, ny, per, 2)
    rhs = torch.tensor(W.normal_field(nx, ny, 3, per), device="cuda")
    upd = mg.Solver(nx, ny, periodic_y=per, kx=a1, **case["opts"])
    ref = mg.Solver(nx, ny, periodic_y=per, kx=a2, **case["opts"])
    try:
        x1 = torch.zeros_like(rhs)
        upd.solve(rhs, x1, 1e-10, 200)  # a solve on the first operators
        upd.update_coefficients(a2)
        xu, xr = torch.zeros_like(rhs), torch.zeros_like(rhs)
        iu = upd.solve(rhs, xu, 1e-10, 200)
        ir = ref.solve(rhs, xr, 1e-10, 200)
    finally:
        upd.close()
        ref.close()
    assert iu.status == ir.status == mg.MG_OK
    assert iu.cycles == ir.cycles
    assert torch.equal(xu, xr)
    assert not torch.equal(xu, x1)


def test_gradient_solver_matches_per_call_setup():
    """Three gradient steps with a changing coefficient: the handle kept by
    GradientSolver (updated each step) and a fresh handle per step give the
    same u, dL/da and dL/df bit for bit."""
    from paper_0805_3041_amd import autograd as AG

    n = 129
    f, ustar = W.manufactured_sine(n)
    ft = torch.tensor(f, device="cuda")
    us = torch.tensor(1.2 * ustar, device="cuda")
    a0 = _cells(n, n, False, 7)
    with AG.GradientSolver(n, n, tol=1e-12, max_cycles=200) as gs:
        for k in range(3):
            a = a0 * (1.0 + 0.2 * k)
            out = []
            for fn in (lambda aa, ff: gs(aa, ff), lambda aa, ff: AG.solve(aa, ff, tol=1e-12, max_cycles=200)):
                aa = a.clone().requires_grad_(True)
                ff = ft.clone().requires_grad_(True)
                u = fn(aa, ff)
                (0.5 * torch.sum((u - us) ** 2)).backward()
                out.append((u.detach(), aa.grad, ff.grad))
            for p, q in zip(out[0], out[1]):
                assert torch.equal(p, q)


def test_gradient_solver_rejects_stale_backward():
    from paper_0805_3041_amd import autograd as AG

    n = 33
    f, _ = W.manufactured_sine(n)
    ft = torch.tensor(f, device="cuda")
    a = _cells(n, n, False, 8)
    with AG.GradientSolver(n, n) as gs:
        a1 = a.clone().requires_grad_(True)
        u1 = gs(a1, ft)
        gs(a * 2.0, ft)
        with pytest.raises(RuntimeError, match="replaced the operators"):
            u1.sum().backward()


def test_invalid_updates_are_rejected():
    mg = _mg()
    n = 257
    a = _cells(n, n, False, 9)
    s = mg.Solver(n, n, kx=a, smoother="gs4c")
    c = mg.Solver(65, 65, eps_x=0.5)
    b = mg.BatchedSolver([(33, 33)], [1.0])
    try:
        bad = a.clone()
        bad[3, 5] = -1.0
        with pytest.raises(mg.MGError) as e:
            s.update_coefficients(bad)
        assert e.value.status == mg.MG_EINVAL
        with pytest.raises(mg.MGError) as e:
            s.update_coefficients(a, a * 2.0)  # one array at setup, two now
        assert e.value.status == mg.MG_EINVAL
        with pytest.raises(mg.MGError) as e:
            c.update_coefficients(_cells(65, 65, False, 1))
        assert e.value.status == mg.MG_EINVAL
        coeffs = mg.mg_coeffs(mg.MG_COEF_CELL9, 0.0, 0.0, a.data_ptr(), a.data_ptr(), 0)
        with pytest.raises(mg.MGError) as e:
            mg.mg_update_coeffs(b.h, coeffs)
        assert e.value.status == mg.MG_EUNSUPPORTED
        # a valid update after the rejected ones still solves
        s.update_coefficients(a * 3.0)
        rhs = torch.tensor(W.normal_field(n, n, 4), device="cuda")
        x = torch.zeros_like(rhs)
        assert s.solve(rhs, x, 1e-10, 100).status == mg.MG_OK
    finally:
        s.close()
        c.close()
        b.close()
