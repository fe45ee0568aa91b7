"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

Per-cycle parity compares the collected solution after the same number of
cycles (same iterates, different rounding order); converged parity compares
solutions driven to a tight tolerance.  Bars: 1e-12 relative L-inf for FP64;
for the MIXED mode a cycle is an FP32 computation (bar 1e-5 per cycle), and
the refined solution must reach the FP64 bar.
"""
import numpy as np
import pytest

from oracle.core import AXIS, RADIAL, OracleProblem
from paper_1703_07206_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def problem(dim, n, stencil, faces, hetero, a, with_G, seed):
    wl = W.random_problem(dim, n, stencil, faces, seed=seed, hetero=hetero, a=a,
                          dirichlet_values=with_G)
    return wl


def gpu_solve(wl, precision="fp64", **kw):
    from paper_1703_07206_amd import sgml
    prec = sgml.MIXED if precision == "mixed" else sgml.FP64
    plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, dev(wl.sigma), precision=prec)
    u, st = plan.solve(dev(wl.f), dev(wl.G), raise_on_failure=False, precision=prec, **kw)
    torch.cuda.synchronize()
    return host(u), st


def oracle_problem(wl):
    return OracleProblem(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, wl.sigma)


CASES = [
    # dim, n, stencil, faces, heterogeneous sigma, a, Dirichlet values
    (2, 5, AXIS, "DDDD", False, 0.0, False),
    (2, 7, AXIS, "DDNN", False, 0.0, True),
    (2, 8, RADIAL, "DNND", True, -0.3, True),
    (2, 6, AXIS, "NNDD", True, 0.0, True),
    (2, 2, AXIS, "DDDD", False, 0.0, True),
    (3, 2, RADIAL, "DDDDDD", True, -0.5, True),
    (3, 4, RADIAL, "DDDDDD", True, -0.5, True),
    (3, 5, RADIAL, "DDNNNN", False, 0.0, True),
    (3, 5, AXIS, "DDDDDD", True, -0.2, False),
    (3, 4, AXIS, "NDNDDN", True, -0.1, True),
    (3, 6, RADIAL, "DDDDDD", True, -0.5, True),
    (3, 6, RADIAL, "DNDDND", False, -0.3, True),
    (3, 6, AXIS, "NDNDDD", False, 0.0, True),
    # Neumann y+ faces under the last-column (4 x 128) tiles of a 64k + 1 level
    (3, 6, RADIAL, "NNDNND", True, -0.2, True),
    (3, 6, AXIS, "DDDNDN", False, -0.1, False),
]
IDS = [f"{d}d-n{n}-{'rad' if s else 'axis'}-{fc}-{'sig' if h else 'one'}" for d, n, s, fc, h, a, g in CASES]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_per_cycle_parity_fp64(case):
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=100 + n)
    P = oracle_problem(wl)
    for cycles in (1, 3):
        u_or, info = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=cycles)
        u_gpu, st = gpu_solve(wl, tol=0.0, max_cycles=cycles, record_pres=True)
        assert st["cycles"] == cycles
        assert rel_inf(u_gpu, u_or) < 1e-12, (cycles, rel_inf(u_gpu, u_or))
        assert abs(st["relres"] - info["relres"]) <= 1e-10 * info["relres"] + 1e-15
        assert abs(st["norm0"] - info["norm0"]) <= 1e-13 * info["norm0"]


@pytest.mark.parametrize("case", CASES[:4] + CASES[6:8] + CASES[11:13], ids=IDS[:4] + IDS[6:8] + IDS[11:13])
def test_pseudo_residuals_per_visit(case):
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=200 + n)
    P = oracle_problem(wl)
    _, pres_or = P.cycle(wl.f, G=wl.G, with_pres=True)
    _, st = gpu_solve(wl, tol=0.0, max_cycles=1, record_pres=True)
    pres_gpu = np.array(st["pres"])
    assert pres_gpu.shape == pres_or.shape
    assert np.max(np.abs(pres_gpu - pres_or)) <= 1e-11 * np.max(pres_or)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_converged_parity_fp64(case):
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=300 + n)
    u_or, info = oracle_problem(wl).solve(wl.f, G=wl.G, tol=1e-15, max_cycles=400)
    assert info["status"] == 0
    u_gpu, st = gpu_solve(wl, tol=1e-15, max_cycles=400)
    assert st["status"] == 0
    assert rel_inf(u_gpu, u_or) < 1e-12


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[6], CASES[7], CASES[10], CASES[11], CASES[13], CASES[14]],
                         ids=[IDS[1], IDS[2], IDS[6], IDS[7], IDS[10], IDS[11], IDS[13], IDS[14]])
def test_mixed_precision(case):
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=400 + n)
    P = oracle_problem(wl)
    # one FP32 cycle against the FP64 cycle
    u1_or, _ = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=1)
    u1_gpu, _ = gpu_solve(wl, "mixed", tol=0.0, max_cycles=1)
    assert rel_inf(u1_gpu, u1_or) < 1e-5
    # refined to the FP64 accuracy
    u_or, info = P.solve(wl.f, G=wl.G, tol=1e-15, max_cycles=400)
    u_gpu, st = gpu_solve(wl, "mixed", tol=1e-14, max_cycles=400)
    assert st["status"] == 0, st
    assert rel_inf(u_gpu, u_or) < 1e-12


@pytest.mark.parametrize("case", [CASES[2], CASES[6], CASES[9]], ids=[IDS[2], IDS[6], IDS[9]])
def test_residual_entry_point(case):
    from paper_1703_07206_amd import sgml
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=500 + n)
    P = oracle_problem(wl)
    u = np.random.default_rng(1).uniform(-1, 1, P.shape)
    m = P.dirichlet_mask()
    r_or = np.where(m, 0.0, wl.f - P.apply(u))
    plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, dev(wl.sigma))
    r = torch.empty(P.shape, dtype=torch.float64, device="cuda")
    _, rmax, norm0 = plan.residual(dev(wl.f), dev(u), G=dev(wl.G), r=r)
    scale = np.max(np.abs(P.apply(u))) + np.max(np.abs(wl.f))
    assert np.max(np.abs(host(r) - r_or)) < 1e-13 * scale
    assert abs(rmax - np.max(np.abs(r_or))) < 1e-13 * scale
    _, info = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=1)
    assert abs(norm0 - info["norm0"]) <= 1e-13 * info["norm0"]


@pytest.mark.parametrize("dim,n,stencil", [(3, 4, RADIAL), (2, 6, AXIS), (2, 5, RADIAL)])
def test_adjoint_and_coefficient_gradient(dim, n, stencil):
    from paper_1703_07206_amd import sgml
    wl = W.random_problem(dim, n, stencil, "DDDDDD", seed=600 + n, hetero=True, a=-0.5)
    P = oracle_problem(wl)
    m = P.dirichlet_mask()
    ut = np.random.default_rng(7).uniform(-1, 1, P.shape)
    u_or, _ = P.solve(wl.f, G=wl.G, tol=1e-15, max_cycles=400)
    g = np.where(m, 0.0, u_or - ut)
    lam_or, _ = P.solve(g, tol=1e-15, max_cycles=400)
    grad_or = P.coeff_grad(u_or, lam_or)
    plan = sgml.Plan(dim, n, stencil, "DDDDDD", wl.a, dev(wl.sigma))
    lam, st = plan.adjoint(dev(g), tol=1e-15, max_cycles=400)
    assert st["status"] == 0
    assert rel_inf(host(lam), lam_or) < 1e-12
    assert np.all(host(lam)[m] == 0.0)
    grad = plan.coeff_grad(dev(u_or), dev(lam_or))
    assert rel_inf(host(grad), grad_or) < 1e-12


def test_adjoint_rejects_pure_neumann_faces():
    # Neumann faces next to a Dirichlet face are covered (test_gpu_neumann);
    # with no Dirichlet face at all the adjoint is not
    from paper_1703_07206_amd import sgml
    plan = sgml.Plan(2, 4, AXIS, "NNNN")
    g = torch.zeros((17, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(sgml.SGMLError) as ei:
        plan.adjoint(g)
    assert ei.value.status == sgml.E_UNSUPPORTED


def test_schedule_each_tooth_reading():
    wl = problem(2, 6, AXIS, "DDDD", False, 0.0, True, seed=700)
    u_or, _ = oracle_problem(wl).solve(wl.f, G=wl.G, tol=0.0, max_cycles=2, reading=1)
    u_gpu, _ = gpu_solve(wl, tol=0.0, max_cycles=2, schedule=1)
    assert rel_inf(u_gpu, u_or) < 1e-12


@pytest.mark.parametrize("n_r", [1, 3, 0])
def test_relaxation_cap_parity(n_r):
    wl = problem(2, 5, RADIAL, "DDNN", True, 0.0, True, seed=800)
    u_or, _ = oracle_problem(wl).solve(wl.f, G=wl.G, tol=0.0, max_cycles=2, n_r=n_r)
    u_gpu, _ = gpu_solve(wl, tol=0.0, max_cycles=2, n_r=n_r)
    assert rel_inf(u_gpu, u_or) < 1e-12


def test_failure_statuses_and_trivial_problem():
    from paper_1703_07206_amd import sgml
    wl = problem(2, 4, AXIS, "DDDD", False, 0.0, False, seed=900)
    plan = sgml.Plan(2, 4, AXIS, "DDDD", theta=2.5)
    _, st = plan.solve(dev(wl.f), raise_on_failure=False, tol=1e-12, max_cycles=50)
    assert st["status"] == sgml.E_DIVERGED
    plan = sgml.Plan(2, 4, AXIS, "DDDD")
    _, st = plan.solve(dev(wl.f), raise_on_failure=False, tol=1e-12, max_cycles=1)
    assert st["status"] == sgml.E_MAXCYCLES and st["cycles"] == 1
    G = np.random.default_rng(3).uniform(-1, 1, (17, 17))
    # f = 0 with zero Dirichlet values: nothing to do; with values: u = G there
    u, st = plan.solve(dev(np.zeros((17, 17))), tol=1e-12)
    assert st["status"] == 0 and st["cycles"] == 0 and not np.any(host(u))


def test_solves_are_deterministic():
    wl = problem(3, 5, RADIAL, "DDDDDD", True, -0.5, True, seed=1000)
    u1, s1 = gpu_solve(wl, tol=1e-13)
    u2, s2 = gpu_solve(wl, tol=1e-13)
    assert np.array_equal(u1, u2) and s1["history"] == s2["history"]
    m1, _ = gpu_solve(wl, "mixed", tol=1e-13)
    m2, _ = gpu_solve(wl, "mixed", tol=1e-13)
    assert np.array_equal(m1, m2)


@pytest.mark.parametrize("coarse_nodes", [-1, 0, 10 ** 6], ids=["separate", "default", "all-coarse"])
@pytest.mark.parametrize("case", [CASES[2], CASES[3], CASES[7], CASES[9], CASES[10]],
                         ids=[IDS[2], IDS[3], IDS[7], IDS[9], IDS[10]])
def test_coarse_level_kernel_paths(case, coarse_nodes):
    # the same cycle with coarse levels launched one operation at a time, in
    # one workgroup per run of coarse operations, or with every level there
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=1100 + n)
    P = oracle_problem(wl)
    u_or, _ = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=2)
    _, pres_or = P.cycle(wl.f, G=wl.G, with_pres=True)
    for prec, bar in (("fp64", 1e-12), ("mixed", 1e-5)):
        u_gpu, st = gpu_solve(wl, prec, tol=0.0, max_cycles=2, coarse_nodes=coarse_nodes)
        assert rel_inf(u_gpu, u_or) < bar, (prec, rel_inf(u_gpu, u_or))
    _, st = gpu_solve(wl, tol=0.0, max_cycles=1, record_pres=True, coarse_nodes=coarse_nodes)
    assert np.max(np.abs(np.array(st["pres"]) - pres_or)) <= 1e-11 * np.max(pres_or)


FUSED_CASES = [
    (2, 9, AXIS, "DDNN", False, 0.0, True),
    (2, 9, RADIAL, "DNND", True, -0.3, True),
    (2, 8, AXIS, "NNDD", True, 0.0, False),
    (2, 8, RADIAL, "NDDN", False, -0.1, True),
]
FUSED_IDS = [f"n{n}-{'rad' if s else 'axis'}-{fc}-{'sig' if h else 'one'}" for d, n, s, fc, h, a, g in FUSED_CASES]


@pytest.mark.parametrize("n_r,sched", [(2, 0), (1, 0), (3, 0), (2, 1), (0, 0)],
                         ids=["nr2", "nr1", "nr3", "nr2-each", "full-doubling"])
@pytest.mark.parametrize("case", FUSED_CASES, ids=FUSED_IDS)
def test_fused_visits_match_oracle(case, n_r, sched):
    # one pass per visit on the large 2D levels (interpolation prologue,
    # several relaxations, injection epilogue) against the oracle, and
    # against the unfused launches
    dim, n, stencil, faces, hetero, a, with_G = case
    # (full doubling at 513^2: about 5 s per literal oracle cycle on 8 threads)
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=1200 + n)
    P = oracle_problem(wl)
    u_or, info = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=2, n_r=n_r, reading=sched)
    _, pres_or = P.cycle(wl.f, G=wl.G, n_r=n_r, reading=sched, with_pres=True)
    for fuse in (64, -1):
        u, st = gpu_solve(wl, tol=0.0, max_cycles=2, n_r=n_r, schedule=sched, fuse=fuse)
        assert rel_inf(u, u_or) < 1e-12, (fuse, rel_inf(u, u_or))
        um, _ = gpu_solve(wl, "mixed", tol=0.0, max_cycles=2, n_r=n_r, schedule=sched, fuse=fuse)
        assert rel_inf(um, u_or) < 1e-5
        _, st1 = gpu_solve(wl, tol=0.0, max_cycles=1, n_r=n_r, schedule=sched, fuse=fuse,
                           record_pres=True)
        assert np.max(np.abs(np.array(st1["pres"]) - pres_or)) <= 1e-11 * np.max(pres_or)


@pytest.mark.parametrize("case", [FUSED_CASES[0], FUSED_CASES[3]], ids=[FUSED_IDS[0], FUSED_IDS[3]])
def test_fused_cycle_end_same_results(case):
    # FP32 cycles with the closing level-0 visit (interpolation and six
    # relaxations at n_r = 2) and the cycle end in one pass, forced on these
    # small grids, give the results of the two passes cycle by cycle, and the
    # oracle's within the FP32 bar
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=1250 + n)
    u_or, _ = oracle_problem(wl).solve(wl.f, G=wl.G, tol=0.0, max_cycles=3)
    u1, st1 = gpu_solve(wl, "mixed", tol=0.0, max_cycles=3, fuse_end=1)
    u0, st0 = gpu_solve(wl, "mixed", tol=0.0, max_cycles=3, fuse_end=-1)
    assert np.array_equal(u1, u0) and st1["history"] == st0["history"]
    assert rel_inf(u1, u_or) < 1e-5
    # the fused pass ran in the cycles after the first (the first imposes G)
    _, sp = gpu_solve(wl, "mixed", tol=0.0, max_cycles=3, fuse_end=1, profile=True)
    assert sp["prof"]["visit0_end"]["launches"] == (2 if with_G else 3)
    _, sp = gpu_solve(wl, "mixed", tol=0.0, max_cycles=3, fuse_end=-1, profile=True)
    assert sp["prof"]["visit0_end"]["launches"] == 0


@pytest.mark.parametrize("case", FUSED_CASES[:2], ids=FUSED_IDS[:2])
def test_fused_visits_converged(case):
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=1300 + n)
    u_or, _ = oracle_problem(wl).solve(wl.f, G=wl.G, tol=1e-15, max_cycles=200)
    for prec, tol in (("fp64", 1e-15), ("mixed", 1e-14)):
        u, st = gpu_solve(wl, prec, tol=tol, max_cycles=200, fuse=64)
        assert st["status"] == 0
        assert rel_inf(u, u_or) < 1e-12


@pytest.mark.parametrize("case", [(2, 10, AXIS, "DDNN", False, 0.0, True), (2, 10, RADIAL, "NDDN", True, -0.2, True)],
                         ids=["n10-axis-DDNN-one", "n10-rad-NDDN-sig"])
def test_per_cycle_parity_1025(case):
    # every 2D kernel of the default path at once: the row-marching visits of
    # levels 0..3 (1025^2..129^2), the coarse levels in LDS, and the cycle end
    # (mixed: with the level-1 restriction)
    dim, n, stencil, faces, hetero, a, with_G = case
    wl = problem(dim, n, stencil, faces, hetero, a, with_G, seed=1500 + n)
    P = oracle_problem(wl)
    u_or, info = P.solve(wl.f, G=wl.G, tol=0.0, max_cycles=2)
    u, st = gpu_solve(wl, tol=0.0, max_cycles=2)
    assert rel_inf(u, u_or) < 1e-12, rel_inf(u, u_or)
    assert abs(st["relres"] - info["relres"]) <= 1e-10 * info["relres"]
    um, stm = gpu_solve(wl, "mixed", tol=0.0, max_cycles=2)
    assert rel_inf(um, u_or) < 1e-5, rel_inf(um, u_or)
    # refined to the FP64 bar against the oracle's converged solution
    u_or_c, _ = P.solve(wl.f, G=wl.G, tol=1e-13, max_cycles=60)
    umc, stc = gpu_solve(wl, "mixed", tol=1e-13, max_cycles=60)
    assert stc["status"] == 0
    assert rel_inf(umc, u_or_c) < 1e-12, rel_inf(umc, u_or_c)
