"""The no-allocation entry point (sgml_solve_noalloc) against sgml_solve.

Two calls in a row on one device, the second with a smaller input, both
compared with the ordinary entry point on the same inputs (FP64 bar 1e-12
relative L-inf; the kernels and their order are the same, so the results
are expected to be identical), plus the refusal of a problem whose
workspace exceeds the static one.
"""
import numpy as np
import pytest

from oracle.core import AXIS, RADIAL
from paper_1703_07206_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel_inf(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_solve_on_two_calls(precision):
    from paper_1703_07206_amd import sgml
    prec = sgml.MIXED if precision == "mixed" else sgml.FP64
    big = W.random_problem(2, 9, RADIAL, "DDNN", seed=41, hetero=True, a=-0.2)
    small = W.random_problem(3, 5, AXIS, "NDDDDN", seed=42, hetero=True, a=-0.1)
    results = []
    for wl in (big, small):
        # the ordinary plan (own workspace) and a plan without workspace
        ref_plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, dev(wl.sigma), precision=prec)
        na_plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, dev(wl.sigma), precision=prec,
                            workspace=False)
        f, G = dev(wl.f), dev(wl.G)
        u_ref, st_ref = ref_plan.solve(f, G, tol=1e-13, max_cycles=200, precision=prec)
        u = torch.full_like(f, float("nan"))
        na_plan.solve_noalloc(f, G, u, tol=1e-13, max_cycles=200, precision=prec)
        # a plan with a workspace may use the static one as well
        u2 = torch.full_like(f, float("nan"))
        _, st2 = ref_plan.solve_noalloc(f, G, u2, tol=1e-13, max_cycles=200, precision=prec)
        torch.cuda.synchronize()
        results.append((rel_inf(u, u_ref), rel_inf(u2, u_ref), st2["cycles"], st_ref["cycles"]))
    for e1, e2, c1, c2 in results:
        assert e1 < 1e-12 and e2 < 1e-12, results
        assert c1 == c2, results


def test_noalloc_refuses_problems_beyond_its_workspace():
    from paper_1703_07206_amd import sgml
    plan = sgml.Plan(2, 11, AXIS, "DDDD", workspace=False)  # 2049^2 FP64: 140 MiB
    assert plan.workspace_bytes > 64 << 20
    f = torch.zeros((2049, 2049), dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    with pytest.raises(sgml.SGMLError) as ei:
        plan.solve_noalloc(f, None, u)
    assert ei.value.status == sgml.E_WORKSPACE
    # a plan without workspace refuses the entry points that need one
    with pytest.raises(sgml.SGMLError) as ei:
        plan.solve(f, None, u)
    assert ei.value.status == sgml.E_WORKSPACE
    with pytest.raises(sgml.SGMLError) as ei:
        plan.solve_noalloc(f, None, u, profile=True)
    assert ei.value.status == sgml.E_ARG
