"""GPU parity on spherical coordinates (coefficients r^2 sin(theta) and
sin(theta), different per-cell kx and ky varying in both directions): per
cycle against the oracle for point and line smoothers, on a finest level run
by the coarse-level interpreter and on one whose kernels form the couplings
from the two cell arrays; the mixed form reaches the tolerance."""

import numpy as np
import pytest

import workloads as W
from tests.problems import Problem
from tests.test_gpu_parity import check_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("smoother", ["gs4c", "gstri_x", "gsadi", "tri_x"])
@pytest.mark.parametrize("n,cta", [(65, 0), (129, 300)])
def test_sphere_per_cycle(n, cta, smoother):
    p = Problem(n, n, q1="sphere", smoother=smoother, omega=0.8)
    check_parity(p, W.normal_field(n, n, 3), W.uniform_field(n, n, 1), 3, coarse_cta_nodes=cta)


def test_sphere_mixed_precision_reaches_tolerance():
    from oracle import mg_oracle as O
    n = 257
    p = Problem(n, n, q1="sphere", smoother="gsadi")
    g = p.grid()
    rhs = W.normal_field(n, n, 3)
    s = p.solver(precision="mixed")
    try:
        x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        info = s.solve(torch.tensor(rhs, device="cuda"), x, tol=1e-10, max_cycles=100)
    finally:
        s.close()
    assert info.status == 0 and info.cycles <= 12
    h = p.oracle()
    b = g.pack(rhs)
    rel = O.residual_norm(h, b, g.pack(x.cpu().numpy())) / O.residual_norm(h, b, np.zeros_like(b))
    assert rel <= 1e-10
