"""GPU parity of the Neumann-face extensions against the FP64 oracle.

* The adjoint with Neumann faces (transposed solve through the trapezoid
  weights) and the coefficient gradient with node images: the paper's own
  heterogeneous problem of Sec. 3.4 (eq. 15-16, Neumann lateral faces) at
  129^3 against central finite differences, and small grids against the
  oracle's adjoint and gradient.
* Pure Neumann problems (Sec. 2, last paragraph; Sec. 3.2 eq. 10): per-cycle
  and converged parity, and the circle-source potential of Sec. 3.2 against
  its exact discrete (DCT-I) solution.
* Neumann data moved to the source (Sec. 2): the library's source against the
  oracle's, and a quadratic reproduced exactly.
Bars: FP64 1e-12 relative L-inf; gradients 1e-6 against central differences.
"""
import numpy as np
import pytest

from oracle import exact
from oracle.core import AXIS, RADIAL, OracleProblem
from paper_1703_07206_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def oracle_problem(wl):
    return OracleProblem(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, wl.sigma)


def plan_for(wl, precision=None):
    from paper_1703_07206_amd import sgml
    return sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, dev(wl.sigma),
                     precision=sgml.MIXED if precision is None else precision)


def trap_mean(v, faces):
    dim = v.ndim
    w = np.ones(v.shape)
    for ax in range(dim):
        arr_ax = dim - 1 - ax
        for side, pos in ((faces[2 * ax], 0), (faces[2 * ax + 1], v.shape[0] - 1)):
            if side == "N":
                sl = [slice(None)] * dim
                sl[arr_ax] = pos
                w[tuple(sl)] *= 0.5
    return np.sum(w * v) / np.sum(w)


# ------------------------------------------------------------- adjoint

ADJ_CASES = [
    (2, 5, RADIAL, "DDNN"), (2, 6, AXIS, "NDND"), (2, 8, RADIAL, "NNND"),
    (3, 4, RADIAL, "NNNNDD"), (3, 5, AXIS, "DNDNND"), (3, 6, RADIAL, "NNNNDD"),
]
ADJ_IDS = [f"{d}d-n{n}-{'rad' if s else 'axis'}-{fc}" for d, n, s, fc in ADJ_CASES]


@pytest.mark.parametrize("case", ADJ_CASES, ids=ADJ_IDS)
def test_adjoint_and_gradient_with_neumann_faces(case):
    from paper_1703_07206_amd import sgml
    dim, n, stencil, faces = case
    wl = W.random_problem(dim, n, stencil, faces, seed=1800 + n, hetero=True, a=-0.3)
    P = oracle_problem(wl)
    m = P.dirichlet_mask()
    rng = np.random.default_rng(1801)
    g = np.where(m, 0.0, rng.uniform(-1, 1, P.shape))
    lam_or, info = P.adjoint(g, tol=1e-15, max_cycles=400)
    assert info["status"] == 0
    plan = plan_for(wl)
    for prec, tol in ((sgml.FP64, 1e-15), (sgml.MIXED, 1e-14)):
        lam, st = plan.adjoint(dev(g), tol=tol, max_cycles=400, precision=prec)
        assert st["status"] == 0
        lh = host(lam)
        assert rel_inf(lh, lam_or) < 1e-12, (prec, rel_inf(lh, lam_or))
        assert np.all(lh[m] == 0.0)
    # the gradient kernel on the same inputs, element by element
    u = rng.uniform(-1, 1, P.shape)
    grad = plan.coeff_grad(dev(u), dev(lam_or))
    assert rel_inf(host(grad), P.coeff_grad(u, lam_or)) < 1e-12


def test_adjoint_rejects_pure_neumann_problems():
    from paper_1703_07206_amd import sgml
    plan = sgml.Plan(2, 4, AXIS, "NNNN", a=0.1)
    g = torch.zeros((17, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(sgml.SGMLError) as ei:
        plan.adjoint(g)
    assert ei.value.status == sgml.E_UNSUPPORTED


def _loss(u, ut, mask):
    d = np.where(mask, 0.0, u - ut)
    return 0.5 * np.sum(d * d)


@pytest.mark.parametrize("sign", [1, -1])
def test_capacitor_tanh_gradients_sec34(sign):
    # Sec. 3.4 (eq. 15-16, Neumann lateral faces): dLoss/df and dLoss/dsigma
    # from the differentiable solve against central finite differences at
    # 129^3, and against the oracle's adjoint gradient at 33^3
    from paper_1703_07206_amd import sgml
    from paper_1703_07206_amd.autograd import SGMLSolve
    small = W.capacitor_tanh(n=5, sign=sign)
    Ps = oracle_problem(small)
    ms = Ps.dirichlet_mask()
    uts = W.smooth_target(5, np.random.default_rng(1900))
    u_or, _ = Ps.solve(small.f, G=small.G, tol=1e-15, max_cycles=200)
    lam_or, _ = Ps.adjoint(np.where(ms, 0.0, u_or - uts), tol=1e-15, max_cycles=200)
    gs_or = Ps.coeff_grad(u_or, lam_or)
    plan = plan_for(small, sgml.FP64)
    f = dev(small.f).requires_grad_(True)
    sig = dev(small.sigma).requires_grad_(True)
    opts = dict(tol=1e-15, max_cycles=200)
    u = SGMLSolve.apply(f, sig, plan, dev(small.G), opts)
    (0.5 * torch.sum(torch.where(torch.from_numpy(ms).cuda(), 0.0, u - dev(uts)) ** 2)).backward()
    assert rel_inf(host(f.grad), lam_or) < 1e-12
    assert rel_inf(host(sig.grad), gs_or) < 1e-12

    wl = W.capacitor_tanh(n=7, sign=sign)
    P = oracle_problem(wl)
    m = P.dirichlet_mask()
    rng = np.random.default_rng(1901)
    ut = W.smooth_target(7, rng)
    plan = plan_for(wl, sgml.FP64)
    opts = dict(tol=1e-14, max_cycles=200)
    f = dev(wl.f).requires_grad_(True)
    sig = dev(wl.sigma).requires_grad_(True)
    G = dev(wl.G)
    u = SGMLSolve.apply(f, sig, plan, G, opts)
    (0.5 * torch.sum(torch.where(torch.from_numpy(m).cuda(), 0.0, u - dev(ut)) ** 2)).backward()
    gf, gs = host(f.grad), host(sig.grad)
    N = wl.N
    # interior picks and nodes of the Neumann lateral faces, edges included
    picks = [tuple(int(v) for v in rng.integers(1, N - 1, 3)) for _ in range(4)]
    picks += [(N // 2, N // 3, 0), (N // 3, 0, N // 2), (2 * N // 3, N - 1, N - 1), (N // 4, 0, 0)]
    base = dict(tol=1e-14, max_cycles=200, precision=sgml.FP64)
    plan.set_coeffs(dev(wl.sigma))
    for node in picks:
        fp, fm = wl.f.copy(), wl.f.copy()
        fp[node] += 1.0
        fm[node] -= 1.0
        up, _ = plan.solve(dev(fp), G, **base)
        um, _ = plan.solve(dev(fm), G, **base)
        fd = (_loss(host(up), ut, m) - _loss(host(um), ut, m)) / 2.0
        assert abs(fd - gf[node]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(gf))), (node, fd, gf[node])
    for node in picks:
        d = 1e-4 * wl.sigma[node]
        res = []
        for sgn in (1, -1):
            sp = wl.sigma.copy()
            sp[node] += sgn * d
            plan.set_coeffs(dev(sp))
            uu, _ = plan.solve(dev(wl.f), G, **base)
            res.append(host(uu))
        dd = np.where(m, 0.0, res[0] - res[1])
        ss = np.where(m, 0.0, res[0] + res[1] - 2 * ut)
        fd = 0.5 * np.sum(dd * ss) / (2 * d)
        assert abs(fd - gs[node]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(gs))), (node, fd, gs[node])


# ------------------------------------------------------------- pure Neumann

PN_CASES = [
    # dim, n, stencil, a, heterogeneous sigma
    (2, 6, RADIAL, 0.1, False), (2, 8, AXIS, 0.0, True), (2, 8, RADIAL, 0.1, True),
    (3, 5, RADIAL, 0.1, False), (3, 6, AXIS, 0.0, True),
]
PN_IDS = [f"{d}d-n{n}-{'rad' if s else 'axis'}-a{a}-{'sig' if h else 'one'}" for d, n, s, a, h in PN_CASES]


@pytest.mark.parametrize("case", PN_CASES, ids=PN_IDS)
def test_pure_neumann_parity(case):
    from paper_1703_07206_amd import sgml
    dim, n, stencil, a, hetero = case
    faces = "N" * (2 * dim)
    wl = W.random_problem(dim, n, stencil, faces, seed=2000 + n, hetero=hetero, a=a)
    P = oracle_problem(wl)
    plan = plan_for(wl)
    for cycles in (1, 3):
        u_or, info = P.solve(wl.f, tol=0.0, max_cycles=cycles, stall_window=-1)
        u, st = plan.solve(dev(wl.f), tol=0.0, max_cycles=cycles, stall_window=-1, precision=sgml.FP64,
                           raise_on_failure=False)
        assert rel_inf(host(u), u_or) < 1e-12, (cycles, rel_inf(host(u), u_or))
        assert abs(st["norm0"] - info["norm0"]) <= 1e-13 * info["norm0"]
        assert abs(st["relres"] - info["relres"]) <= 1e-10 * info["relres"]
    u_or, info = P.solve(wl.f, tol=1e-15, max_cycles=300)
    assert info["status"] == 0
    for prec, tol in ((sgml.FP64, 1e-15), (sgml.MIXED, 1e-14)):
        u, st = plan.solve(dev(wl.f), tol=tol, max_cycles=300, precision=prec)
        assert st["status"] == 0
        uh = host(u)
        assert rel_inf(uh, u_or) < 1e-12, (prec, rel_inf(uh, u_or))
        assert abs(trap_mean(uh, faces)) < 1e-13 * np.max(np.abs(uh))


@pytest.mark.parametrize("n", [6, 7])
def test_neumann_circle_sec32(n):
    # the grid-deformation potential of Sec. 3.2 (65^2 and 129^2, a = 0.1)
    # against its exact discrete solution (DCT-I on both axes)
    from paper_1703_07206_amd import sgml
    wl = W.neumann_circle(n=n)
    fp = wl.f - trap_mean(wl.f, "NNNN")
    ref = exact.spectral_solve(2, n, RADIAL, "NNNN", 0.1, fp)
    plan = plan_for(wl)
    for prec, tol in ((sgml.FP64, 1e-14), (sgml.MIXED, 1e-14)):
        u, st = plan.solve(dev(wl.f), tol=tol, max_cycles=100, precision=prec)
        assert st["status"] == 0 and st["cycles"] <= 20, st["cycles"]
        assert rel_inf(host(u), ref) < 1e-12, (prec, rel_inf(host(u), ref))


# ------------------------------------------------------------- Neumann data

@pytest.mark.parametrize("dim,n,stencil,faces", [(2, 7, RADIAL, "NNDN"), (2, 9, AXIS, "DNNN"),
                                                 (3, 5, RADIAL, "NNNNDN"), (3, 6, AXIS, "DNNNNN")])
def test_neumann_data_source_and_solve(dim, n, stencil, faces):
    from paper_1703_07206_amd import sgml
    wl = W.random_problem(dim, n, stencil, faces, seed=2100 + n, hetero=True, a=-0.2)
    P = oracle_problem(wl)
    N = P.N
    rng = np.random.default_rng(2101)
    flux = [rng.uniform(-1, 1, (N,) * (dim - 1)) for _ in range(2 * dim)]
    ref = P.neumann_source(wl.f, flux)
    plan = plan_for(wl)
    out = plan.neumann_source(dev(wl.f), [dev(g) for g in flux])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(host(out) - ref)) <= 1e-14 * scale
    # the solve with the data against the oracle's
    u_or, _ = P.solve(ref, G=wl.G, tol=1e-15, max_cycles=300)
    u, st = plan.solve(out, dev(wl.G), tol=1e-15, max_cycles=300, precision=sgml.FP64)
    assert st["status"] == 0
    assert rel_inf(host(u), u_or) < 1e-12
