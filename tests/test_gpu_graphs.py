"""Cycles replayed as HIP graphs against the same cycles launched one by one.

Every cycle after the first is a replay of a captured graph, with the host's
own stop test (a synchronisation and a read of the residual norm) between
replays; repeated solves reuse the graph kept by the plan, and a different
output buffer or option set captures a new one.  The results must be
bitwise equal to the eager launches'."""
import numpy as np
import pytest

from oracle.core import AXIS, RADIAL
from paper_1703_07206_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


CASES = [
    # dim, n, stencil, faces, heterogeneous sigma, a, Dirichlet values
    (2, 10, AXIS, "DDNN", False, 0.0, True),     # row-marching visits, double-buffered residual (mixed)
    (2, 8, RADIAL, "DNND", True, -0.3, True),    # row-marching visits with a coefficient, coarse kernel
    (3, 6, RADIAL, "DDDDDD", False, 0.0, True),  # z-marching paired relaxations, LDS cycle end
    (3, 5, AXIS, "NDNDDN", True, -0.2, True),    # single 3D relaxations
    (2, 7, RADIAL, "NNNN", False, 0.1, False),   # pure Neumann projections
]
IDS = [f"{d}d-n{n}-{'rad' if s else 'axis'}-{fc}" for d, n, s, fc, h, a, g in CASES]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_graph_replays_equal_eager_launches(case):
    from paper_1703_07206_amd import sgml
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = W.random_problem(dim, n, stencil, faces, seed=2400 + n, hetero=hetero, a=a, dirichlet_values=with_G)
    plan = sgml.Plan(dim, n, stencil, faces, a, dev(wl.sigma), precision=sgml.MIXED)
    f, G = dev(wl.f), dev(wl.G)
    for prec, tol in ((sgml.FP64, 1e-13), (sgml.MIXED, 1e-13)):
        ref, st_ref = plan.solve(f, G, tol=tol, max_cycles=200, precision=prec, graphs=-1)
        u = torch.empty_like(f)
        for rep in range(3):  # capture, then replays of the kept graph
            u.fill_(float("nan"))
            _, st = plan.solve(f, G, u, tol=tol, max_cycles=200, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(u, ref), (prec, rep)
            assert st["history"] == st_ref["history"]
        # another output buffer and the per-visit pseudo-residuals: a new capture
        u2, st2 = plan.solve(f, G, tol=tol, max_cycles=200, precision=prec, record_pres=True)
        _, st3 = plan.solve(f, G, tol=tol, max_cycles=200, precision=prec, record_pres=True, graphs=-1)
        torch.cuda.synchronize()
        assert torch.equal(u2, ref) and st2["pres"] == st3["pres"]


@pytest.mark.parametrize("stencil", [AXIS, RADIAL], ids=["axis", "rad"])
def test_graph_replays_with_fused_cycle_end(stencil):
    # the closing level-0 visit fused with the cycle end (forced at 513^2)
    # alternates the FP32 source between two buffers, as the residual: one
    # graph per buffer; replays equal the eager launches and the unfused cycle
    from paper_1703_07206_amd import sgml
    wl = W.random_problem(2, 9, stencil, "DDNN", seed=2450, hetero=False, a=0.0, dirichlet_values=True)
    plan = sgml.Plan(2, 9, stencil, "DDNN", 0.0, None, precision=sgml.MIXED)
    f, G = dev(wl.f), dev(wl.G)
    kw = dict(tol=1e-13, max_cycles=200, precision=sgml.MIXED)
    ref, st_ref = plan.solve(f, G, graphs=-1, fuse_end=1, **kw)
    unfused, st_un = plan.solve(f, G, graphs=-1, fuse_end=-1, **kw)
    torch.cuda.synchronize()
    assert torch.equal(ref, unfused) and st_ref["history"] == st_un["history"]
    u = torch.empty_like(f)
    for rep in range(3):
        u.fill_(float("nan"))
        _, st = plan.solve(f, G, u, fuse_end=1, **kw)
        torch.cuda.synchronize()
        assert torch.equal(u, ref), rep
        assert st["history"] == st_ref["history"]


def test_graph_replays_in_batches():
    from paper_1703_07206_amd import sgml
    wls = [W.random_problem(3, 6, RADIAL, "DDDDDD", seed=2500 + r, hetero=False) for r in range(3)]
    F = dev(np.stack([w.f for w in wls]))
    plan = sgml.Plan(3, 6, RADIAL, "DDDDDD", 0.0, None, precision=sgml.MIXED, nrhs=3)
    ref, _ = plan.solve_batch(F, tol=1e-13, max_cycles=100, graphs=-1)
    for _ in range(2):
        U, _ = plan.solve_batch(F, tol=1e-13, max_cycles=100)
        torch.cuda.synchronize()
        assert torch.equal(U, ref)
