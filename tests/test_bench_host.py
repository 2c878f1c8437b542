"""Host-side arithmetic of bench.py's roofline (no GPU): the algorithmic
bytes per node of the finest passes, averaged over the launches of an outer
step of the mixed form, and the digest that ties stored counter summaries
to the kernel sources and compile flags."""

import bench


class _FakeSolver:
    def __init__(self, forms_residual):
        self.forms = forms_residual

    def pass_info(self, level, which):
        assert level == 0 and which == 0
        return {"forms_residual": self.forms}


def test_fp64_pass_bytes_do_not_depend_on_inner_cycles():
    s = _FakeSolver(0)
    assert bench.pass_bytes_per_node(s, "fp64", 0) == 28
    assert bench.pass_bytes_per_node(s, "fp64", 1) == 26
    assert bench.pass_bytes_per_node(s, "fp64", 1, inner=3) == 26


def test_mixed_pass_bytes_one_inner_cycle():
    # pre-pass from e = 0: read r, write e, coarse b and x; with the residual
    # formed in the pass: read the FP64 x and b, write r, e, coarse b and x
    assert bench.pass_bytes_per_node(_FakeSolver(0), "mixed", 0) == 10
    assert bench.pass_bytes_per_node(_FakeSolver(1), "mixed", 0) == 26
    # post-pass adding e into the FP64 iterate
    assert bench.pass_bytes_per_node(_FakeSolver(0), "mixed", 1) == 25


def test_mixed_pass_bytes_average_over_an_outer_step():
    # three inner cycles: one launch of the first/last kind, two plain FP32 passes
    assert bench.pass_bytes_per_node(_FakeSolver(0), "mixed", 1, inner=3) == (25 + 2 * 13) / 3
    assert bench.pass_bytes_per_node(_FakeSolver(0), "mixed", 0, inner=3) == (10 + 2 * 14) / 3
    assert bench.pass_bytes_per_node(_FakeSolver(1), "mixed", 0, inner=3) == (26 + 2 * 14) / 3


def test_digest_covers_flags_and_sources():
    from paper_0805_3041_amd import build

    d = bench.source_digest()
    assert d[:16] == build.source_digest()
    assert "-I" not in build.flags_key().split()  # include paths differ between machines
    assert "--offload-arch=gfx950" in build.flags_key()
