"""Seeded synthetic inputs for the SGML solver.

This module holds no part of the solver's arithmetic: it only draws the
right-hand sides, coefficients and boundary values of the problems below,
with numpy's PCG64 (``numpy.random.default_rng(seed)``), in FP64, on the
host.  The same arrays feed the GPU library and the CPU oracle.

Every problem is returned in the paper's form L(u) = f with
L = div(sigma grad) + a on [0,1]^d, N = 2^n + 1 nodes per axis, arrays
indexed [j, i] (2D) or [k, j, i] (3D) with i along x.  A Poisson problem
-lap(u) = f is therefore handed over with source -f.

Workloads (shaped like the paper's 2D Poisson and 3D heterogeneous
Helmholtz-Poisson examples):

``poisson2d_sine``   129^2, 5-point, Dirichlet 0, f = 2 pi^2 sin sin + 0.1 U(-1,1)
``poisson2d_blobs``  4097^2, 5-point, Dirichlet x-walls / Neumann y-walls,
                     64 Gaussian blobs (width 0.01-0.05, amplitude U(-1,1))
``helmholtz3d_spheres`` 257^3, radial 27-point, eps = 1 with 32 spheres of
                     eps in [2, 80], a = -0.5, f = 0, u = -1 / +1 on z = 0 / 1
``helmholtz3d_adjoint`` 129^3, same medium, f = U(-1,1), loss target u_t
``poisson3d_charges``   513^3, radial 27-point, Dirichlet 0, 256 Gaussian
                     point charges of width 2h plus 1e-3 U(-1,1) noise
``neumann_circle``   65^2 / 129^2, the grid-deformation potential of Sec. 3.2:
                     a = 0.1, zero normal derivative on every face, a delta source
                     on a circle built from tensor hats
``trifoil_vortex``   257^3, the vector Poisson problem of Sec. 3.3: three
                     right-hand sides (a vortex line on the trifoil knot, eq. 13)
``capacitor_tanh``   129^3, the heterogeneous Laplace problem of Sec. 3.4:
                     sigma = 0.55 +/- 0.45 tanh((r - 0.2)/0.1) (eq. 16), u = +1 on
                     the top and -1 on the bottom face, Neumann lateral faces
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

AXIS, RADIAL = 0, 1


@dataclass
class Workload:
    name: str
    dim: int
    n: int
    stencil: int
    faces: str            # 'D'/'N' for x-, x+, y-, y+, z-, z+
    a: float
    f: np.ndarray         # source of L(u) = f
    sigma: Optional[np.ndarray] = None
    G: Optional[np.ndarray] = None   # Dirichlet values (read at Dirichlet nodes only)
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return 2 ** self.n + 1

    @property
    def nodes(self):
        return self.N ** self.dim


def dirichlet_mask(dim, n, faces):
    """Boolean array of the nodes on Dirichlet faces (faces: 'D'/'N' for
    x-, x+, y-, y+, z-, z+), in array order."""
    N = 2 ** n + 1
    m = np.zeros((N,) * dim, bool)
    faces = (faces + "DDDDDD")[:6]
    for ax in range(dim):
        arr_ax = dim - 1 - ax
        for side, pos in ((faces[2 * ax], 0), (faces[2 * ax + 1], N - 1)):
            if side == "D":
                sl = [slice(None)] * dim
                sl[arr_ax] = pos
                m[tuple(sl)] = True
    return m


def coords(n, dim):
    """Node coordinates x_i = i h, returned in array order (z, y, x)."""
    N = 2 ** n + 1
    x = np.linspace(0.0, 1.0, N)
    return np.meshgrid(*([x] * dim), indexing="ij")


def poisson2d_sine(n=7, seed=1, noise=0.1):
    N = 2 ** n + 1
    rng = np.random.default_rng(seed)
    eta = rng.uniform(-1.0, 1.0, (N, N))
    Y, X = coords(n, 2)
    f = 2.0 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y) + noise * eta
    return Workload("poisson2d_sine", 2, n, AXIS, "DDDD", 0.0, -f)


def manufactured2d(n=10):
    """Sec. 3.1: lap(u) = f on the unit square, u = 0 on the boundary, with the
    closed-form solution u = -x^2 y^2 (1 - x^2)(1 - y^2) (eq. 7) and its source
    (eq. 8); 5-point stencil.  The exact continuous solution is returned in
    extra["u_exact"].  No random draws."""
    Y, X = coords(n, 2)
    u = -X ** 2 * Y ** 2 * (1 - X ** 2) * (1 - Y ** 2)
    f = -2.0 * (Y ** 2 * (1 - 6 * X ** 2) * (1 - Y ** 2) + X ** 2 * (1 - 6 * Y ** 2) * (1 - X ** 2))
    return Workload("manufactured2d", 2, n, AXIS, "DDDD", 0.0, f, extra=dict(u_exact=u))


def _blobs2d(n, centers, widths, amps):
    N = 2 ** n + 1
    x = np.linspace(0.0, 1.0, N)
    f = np.zeros((N, N))
    for (cx, cy), s, A in zip(centers, widths, amps):
        gx = np.exp(-((x - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((x - cy) ** 2) / (2.0 * s * s))
        f += A * np.outer(gy, gx)  # separable: exp(-|x-c|^2/2s^2) = gx(x) gy(y)
    return f


def poisson2d_blobs(n=12, seed=2, nblobs=64):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (nblobs, 2))
    s = rng.uniform(0.01, 0.05, nblobs)
    A = rng.uniform(-1.0, 1.0, nblobs)
    f = _blobs2d(n, c, s, A)
    return Workload("poisson2d_blobs", 2, n, AXIS, "DDNN", 0.0, -f)


def sphere_medium(n, seed=3, nspheres=32, eps_lo=2.0, eps_hi=80.0):
    """eps = 1 with spheres painted in draw order (later spheres win) at the
    nodes with |x - c| <= r."""
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (nspheres, 3))
    r = rng.uniform(0.03, 0.15, nspheres)
    e = rng.uniform(eps_lo, eps_hi, nspheres)
    eps = np.ones((N, N, N))
    for (cx, cy, cz), rr, ee in zip(c, r, e):
        lo = [max(0, int(np.floor((q - rr) / h))) for q in (cx, cy, cz)]
        hi = [min(N - 1, int(np.ceil((q + rr) / h))) for q in (cx, cy, cz)]
        zi = np.arange(lo[2], hi[2] + 1)
        yi = np.arange(lo[1], hi[1] + 1)
        xi = np.arange(lo[0], hi[0] + 1)
        Z, Y, X = np.meshgrid(zi * h, yi * h, xi * h, indexing="ij")
        inside = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 <= rr * rr
        sub = eps[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[inside] = ee
    return eps


def capacitor_bc(n):
    """u = -1 on the z = 0 face and +1 on the z = 1 face (their edges
    included), 0 on the other faces."""
    N = 2 ** n + 1
    G = np.zeros((N, N, N))
    G[0] = -1.0
    G[-1] = 1.0
    return G


def helmholtz3d_spheres(n=8, seed=3, k=0.5):
    N = 2 ** n + 1
    eps = sphere_medium(n, seed)
    return Workload("helmholtz3d_spheres", 3, n, RADIAL, "DDDDDD", -k, np.zeros((N, N, N)),
                    sigma=eps, G=capacitor_bc(n))


def smooth_target(n, rng, modes=8):
    """u_t = sum_j b_j prod_i sin(m_ji pi x_i), m in {1,2,3}, b ~ U(-1,1),
    evaluated as outer products of the 1D factors."""
    m = rng.integers(1, 4, (modes, 3))
    b = rng.uniform(-1.0, 1.0, modes)
    N = 2 ** n + 1
    x = np.linspace(0.0, 1.0, N)
    ut = np.zeros((N, N, N))
    for (mx, my, mz), bb in zip(m, b):
        yx = np.multiply.outer(np.sin(my * np.pi * x), bb * np.sin(mx * np.pi * x))
        ut += np.multiply.outer(np.sin(mz * np.pi * x), yx)
    return ut


def helmholtz3d_adjoint(n=7, seed_eps=3, seed=4, k=0.5, n_fd=10):
    N = 2 ** n + 1
    eps = sphere_medium(n, seed_eps)
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, (N, N, N))
    ut = smooth_target(n, rng)
    fd_f = rng.integers(1, N - 1, (n_fd, 3))     # (k, j, i) interior picks
    fd_eps = rng.integers(1, N - 1, (n_fd, 3))
    return Workload("helmholtz3d_adjoint", 3, n, RADIAL, "DDDDDD", -k, f, sigma=eps,
                    G=capacitor_bc(n), extra=dict(u_target=ut, fd_f=fd_f, fd_eps=fd_eps))


def poisson3d_charges(n=9, seed=5, ncharges=256, noise=1e-3, cutoff=8.0):
    """Gaussian charges of width w = 2h, evaluated exactly inside a cube of
    half-side cutoff*w around each centre (beyond it exp(-cutoff^2/2) ~ 1e-14)."""
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    w = 2.0 * h
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (ncharges, 3))
    A = rng.uniform(-1.0, 1.0, ncharges)
    f = noise * rng.uniform(-1.0, 1.0, (N, N, N))
    R = int(np.ceil(cutoff * w / h))
    for (cx, cy, cz), amp in zip(c, A):
        ic = [int(round(q / h)) for q in (cx, cy, cz)]
        lo = [max(0, q - R) for q in ic]
        hi = [min(N - 1, q + R) for q in ic]
        gx = np.exp(-((np.arange(lo[0], hi[0] + 1) * h - cx) ** 2) / (2 * w * w))
        gy = np.exp(-((np.arange(lo[1], hi[1] + 1) * h - cy) ** 2) / (2 * w * w))
        gz = np.exp(-((np.arange(lo[2], hi[2] + 1) * h - cz) ** 2) / (2 * w * w))
        f[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += amp * np.einsum(
            "k,j,i->kji", gz, gy, gx)
    ut = smooth_target(n, rng)
    return Workload("poisson3d_charges", 3, n, RADIAL, "DDDDDD", 0.0, -f,
                    extra=dict(u_target=ut))


def trifoil_vortex(n=8, r=0.2):
    """Sec. 3.3, eq. 12-13: the vector Poisson problem lap(psi) = -omega for a
    singular vortex line on the trifoil knot x(t) = r (sin t + 2 sin 2t,
    cos t - 2 cos 2t, -2 sin 3t), r = 0.2, in the unit box: three right-hand
    sides (f[c] = -omega_c, c = x, y, z) with one operator, psi = 0 on every
    face, radial 27-point stencil.  The curve is centred on the box centre by
    its bounding box and sampled at arc-length steps of about h; each sample
    deposits its tangent increment dx(t) as a tensor product of hat functions
    of half-width h (unit integral); samples whose cell leaves the box are
    dropped.  No random draws."""
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    fine = np.linspace(0.0, 2 * np.pi, 20001)
    curve = lambda t: np.stack([r * (np.sin(t) + 2 * np.sin(2 * t)), r * (np.cos(t) - 2 * np.cos(2 * t)),  # noqa
                                -2 * r * np.sin(3 * t)], axis=-1)
    pts = curve(fine)
    length = np.sum(np.linalg.norm(np.diff(pts, axis=0), axis=1))
    centre = 0.5 - 0.5 * (pts.min(axis=0) + pts.max(axis=0))
    npts = int(np.ceil(length / h))
    t = 2 * np.pi * np.arange(npts) / npts
    dt = 2 * np.pi / npts
    x = curve(t) + 0.5 + centre - 0.5
    dx = np.stack([r * (np.cos(t) + 4 * np.cos(2 * t)), r * (-np.sin(t) + 4 * np.sin(2 * t)),
                   -6 * r * np.cos(3 * t)], axis=-1) * dt
    omega = np.zeros((3, N, N, N))
    for (px, py, pz), d in zip(x, dx):
        i0, j0, k0 = int(np.floor(px / h)), int(np.floor(py / h)), int(np.floor(pz / h))
        if min(i0, j0, k0) < 0 or max(i0, j0, k0) > N - 2:
            continue
        fx, fy, fz = px / h - i0, py / h - j0, pz / h - k0
        for dk, wz in ((0, 1 - fz), (1, fz)):
            for dj, wy in ((0, 1 - fy), (1, fy)):
                for di, wx in ((0, 1 - fx), (1, fx)):
                    omega[:, k0 + dk, j0 + dj, i0 + di] += d * (wx * wy * wz / h ** 3)
    return Workload("trifoil_vortex", 3, n, RADIAL, "DDDDDD", 0.0, -omega, extra=dict(components=3))


def capacitor_tanh(n=7, sign=+1):
    """Sec. 3.4: div(sigma grad u) = 0 (eq. 15) with the spherical
    coefficient of eq. 16 centred in the cube, u = -1 / +1 on the bottom /
    top (z = 0 / z = 1) faces and zero normal derivative on the lateral
    faces.  No random draws."""
    N = 2 ** n + 1
    Z, Y, X = coords(n, 3)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    sigma = 0.55 + sign * 0.45 * np.tanh((r - 0.2) / 0.1)
    G = np.zeros((N, N, N))
    G[0] = -1.0
    G[-1] = 1.0
    return Workload("capacitor_tanh", 3, n, RADIAL, "NNNNDD", 0.0, np.zeros((N, N, N)), sigma=sigma, G=G,
                    extra=dict(sign=sign))


def neumann_circle(n=6, a=0.1, radius=0.25, center=(0.5, 0.5)):
    """Sec. 3.2, eq. 10: lap(u) + a u = f - mean(f) with zero normal derivative
    on every face, a = 0.1, f a delta function on a circle: the curve is
    sampled at points one mesh spacing apart (arc length h), and each point
    deposits a tensor product of hat functions of half-width h, normalised to
    unit integral, weighted by its arc length.  Radial 9-point stencil (the
    2D stencil the paper reports convergence with).  No random draws.  The
    mean is removed by the solver."""
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    npts = max(8, int(round(2 * np.pi * radius / h)))
    ds = 2 * np.pi * radius / npts
    t = 2 * np.pi * np.arange(npts) / npts
    f = np.zeros((N, N))
    for px, py in zip(center[0] + radius * np.cos(t), center[1] + radius * np.sin(t)):
        i0, j0 = int(np.floor(px / h)), int(np.floor(py / h))
        fx, fy = px / h - i0, py / h - j0
        for dj, wy in ((0, 1 - fy), (1, fy)):
            for di, wx in ((0, 1 - fx), (1, fx)):
                f[j0 + dj, i0 + di] += ds * wx * wy / (h * h)
    return Workload("neumann_circle", 2, n, RADIAL, "NNNN", a, f)


def random_problem(dim, n, stencil, faces, seed, hetero=True, a=0.0, dirichlet_values=True):
    """Small generic problem for parity tests: random source, smooth positive
    coefficient with random contrast, random Dirichlet values."""
    N = 2 ** n + 1
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, (N,) * dim)
    sigma = np.exp(rng.uniform(-1.0, 1.0, (N,) * dim)) if hetero else None
    G = rng.uniform(-1.0, 1.0, (N,) * dim) if dirichlet_values else None
    return Workload(f"random{dim}d", dim, n, stencil, faces, a, f, sigma=sigma, G=G)


CONFIGS = {
    "poisson2d_sine": poisson2d_sine,
    "poisson2d_blobs": poisson2d_blobs,
    "helmholtz3d_spheres": helmholtz3d_spheres,
    "helmholtz3d_adjoint": helmholtz3d_adjoint,
    "poisson3d_charges": poisson3d_charges,
    "capacitor_tanh": capacitor_tanh,
    "neumann_circle": neumann_circle,
    "manufactured2d": manufactured2d,
    "trifoil_vortex": trifoil_vortex,
}
