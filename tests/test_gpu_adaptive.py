"""Adaptive coarse-correction weight omega_l (the choice "The Multigrid
Technique" allows in place of a fixed value): the energy-minimising weight
of the prolonged correction, computed on every level visit by a reduction
over the level.  GPU iterates against the oracle's cycle with the same
weight, per cycle to 1e-12, through every path that adds a correction:
fused narrow and wide post-passes (the weight read from the level's
descriptor), per-op prolongation, the single-workgroup interpreter in LDS
and in global memory, line smoothers, W- and V-cycles, 9-point operators;
fused equal per-op bit for bit; mixed precision; batched slots equal their
single solves; the nested start; cycles to tolerance."""

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W
from tests.problems import Problem
from tests.test_gpu_parity import PARITY, check_parity, gpu_iterates, oracle_iterates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mg():
    from paper_0805_3041_amd import mg
    return mg


CASES = [
    dict(p=dict(nx=65, ny=65, eps=0.1, smoother="rbgs"), cta=0),                    # LDS interpreter only
    dict(p=dict(nx=129, ny=129, eps=0.1, smoother="rbgs"), cta=300),                # fused passes + interpreter
    dict(p=dict(nx=129, ny=129, eps=0.3, smoother="rbgs"), cta=20000),              # interpreter on global memory
    dict(p=dict(nx=257, ny=257, eps=0.05, smoother="rbgs", nu_pre=1, nu_post=3), cta=300),
    dict(p=dict(nx=97, ny=49, eps=0.3, smoother="rbgs"), cta=100, extra=dict(tile_mode="per_op")),
    dict(p=dict(nx=129, ny=128, periodic_y=True, q1="annulus", smoother="gs4c"), cta=300),
    dict(p=dict(nx=65, ny=64, periodic_y=True, q1="annulus", smoother="gs4c"), cta=0),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c"), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="jacobi", nu_pre=3, nu_post=1), cta=300),
    dict(p=dict(nx=129, ny=129, eps=0.2, smoother="rbgs", cycle="W"), cta=300),
    dict(p=dict(nx=129, ny=129, eps=0.2, smoother="rbgs", cycle="V"), cta=100),
    dict(p=dict(nx=65, ny=65, eps=0.01, smoother="gstri_y"), cta=0),
    dict(p=dict(nx=129, ny=129, eps=0.01, smoother="gsadi"), cta=300),
    dict(p=dict(nx=65, ny=65, eps=1.0, smoother="jacobi", omega=0.8), cta=1),
]


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_adaptive_weight_per_cycle(case):
    p = Problem(adaptive_omega=True, **case["p"])
    check_parity(p, W.normal_field(p.nx, p.ny, 2, p.periodic_y), W.uniform_field(p.nx, p.ny, 1, p.periodic_y), 3,
                 coarse_cta_nodes=case["cta"], **case.get("extra", {}))


def test_adaptive_weight_changes_the_iterate():
    """The weight is not 1 on these levels: the adaptive cycle's iterate
    differs from the fixed-weight one (and each matches its oracle)."""
    n = 129
    rhs = W.normal_field(n, n, 2)
    x0 = np.zeros((n, n))
    out = []
    for adaptive in (False, True):
        s = Problem(n, n, eps=0.1, adaptive_omega=adaptive).solver(coarse_cta_nodes=300)
        try:
            out.append(gpu_iterates(s, rhs, x0, 1)[0])
        finally:
            s.close()
    assert np.abs(out[0] - out[1]).max() > 1e-6 * np.abs(out[0]).max()


WIDE_CASES = [
    dict(p=dict(nx=257, ny=257, eps=0.1, smoother="rbgs"), cta=300),
    dict(p=dict(nx=257, ny=256, periodic_y=True, q1="annulus", smoother="gs4c"), cta=300),
    dict(p=dict(nx=129, ny=129, q1="grf", smoother="gs4c"), cta=300),
]


@pytest.mark.parametrize("mode", ["narrow", "wide"])
@pytest.mark.parametrize("case", WIDE_CASES, ids=[str(i) for i in range(len(WIDE_CASES))])
def test_fused_adaptive_equals_per_op_bitwise(case, mode):
    p = Problem(adaptive_omega=True, **case["p"])
    rhs = W.normal_field(p.nx, p.ny, 21, p.periodic_y)
    x0 = W.uniform_field(p.nx, p.ny, 22, p.periodic_y)
    a = p.solver(coarse_cta_nodes=case["cta"], tile_mode="per_op")
    b = p.solver(coarse_cta_nodes=case["cta"], tile_mode=mode)
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


def test_adaptive_cycles_to_tolerance_equal_oracle():
    n = 129
    p = Problem(n, n, eps=0.1, adaptive_omega=True)
    g = p.grid()
    rhs = W.aniso_rhs(n, 2)
    ref = O.solve(p.oracle(), g.pack(rhs), np.zeros(g.n_unknowns), 1e-10, 500)
    s = p.solver(coarse_cta_nodes=300)
    try:
        x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        info = s.solve(torch.tensor(rhs, device="cuda"), x, 1e-10, 500)
    finally:
        s.close()
    assert ref.status == O.OK and info.status == 0
    assert info.cycles == ref.cycles, (info.cycles, ref.cycles)


def test_adaptive_mixed_precision():
    """FP32 cycles with the adaptive weight: the first outer step within FP32
    rounding of the oracle's mixed form (1e-5), and the solve reaches 1e-10 by
    the oracle's FP64 residual."""
    n = 129
    p = Problem(n, n, eps=0.1, adaptive_omega=True)
    g = p.grid()
    h = p.oracle()
    rhs = W.aniso_rhs(n, 2)
    b = g.pack(rhs)
    one = O.solve_mixed(h, b, np.zeros(g.n_unknowns), 1e-300, 1)
    s = p.solver(precision="mixed", coarse_cta_nodes=300)
    try:
        r = torch.tensor(rhs, device="cuda")
        x = torch.zeros_like(r)
        s.solve(r, x, 1e-300, 1, history=False)
        err = np.abs(g.pack(x.cpu().numpy()) - one.x).max() / np.abs(one.x).max()
        assert err <= 1e-5, err
        x.zero_()
        info = s.solve(r, x, 1e-10, 300)
        xs = x.cpu().numpy()
    finally:
        s.close()
    assert info.status == 0
    assert O.residual_norm(h, b, g.pack(xs)) <= 1.0001e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adaptive_batched_equals_single_solves(precision):
    mg = _mg()
    sizes = [33, 65, 129, 65, 257]
    eps = [1.0, 0.3, 0.05, 1e-2, 0.2]
    rhs = [torch.tensor(W.normal_field(n, n, 1000 + i), device="cuda") for i, n in enumerate(sizes)]
    B = mg.BatchedSolver([(n, n) for n in sizes], eps, smoother="rbgs", precision=precision, adaptive_omega=True)
    xb = [torch.zeros_like(r) for r in rhs]
    outs = []
    try:
        for _ in range(2):
            B.solve(rhs, xb, 1e-300, 1)
            outs.append([x.cpu().numpy().copy() for x in xb])
    finally:
        B.close()
    for i, (n, e) in enumerate(zip(sizes, eps)):
        s = mg.Solver(n, n, eps_x=e, smoother="rbgs", precision=precision, adaptive_omega=True)
        x = torch.zeros_like(rhs[i])
        try:
            for c in range(2):
                s.solve(rhs[i], x, 1e-300, 1, history=False)
                assert np.array_equal(x.cpu().numpy(), outs[c][i]), (i, c)
        finally:
            s.close()


def test_adaptive_nested_start_matches_oracle():
    p = Problem(129, 129, eps=0.1, adaptive_omega=True)
    g = p.grid()
    rhs = p.rhs(5)
    want = O.nested_start(p.oracle(), g.pack(rhs))
    s = p.solver(coarse_cta_nodes=300)
    try:
        r = torch.tensor(rhs, device="cuda")
        x = torch.full_like(r, 3.0)
        s.nested_start(r, x)
        err = np.abs(g.pack(x.cpu().numpy()) - want).max() / np.abs(want).max()
    finally:
        s.close()
    assert err <= PARITY, err
