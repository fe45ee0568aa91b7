"""Exact discrete solutions that pin the oracle -- TEST INFRASTRUCTURE.

Nothing here runs the SGML method.  These are textbook/library routes to
the algebraic solution of dL(u) = f, written independently of the C
oracle's neighbour loop:

* ``kron_apply``     -- the sigma = 1 operators written as sums of products
  of 1D second differences T (one per axis; Neumann faces by node images).
  The axis stencil is sum_i T_i / h^2.  The radial stencil of eq. (5) with
  the 1/l^2 reading expands, over the neighbour classes (faces, edges,
  corners), to
      2D: (T_x + T_y + T_x T_y / 4) / h^2
      3D: (sum T_i + 7/26 sum_{i<j} T_i T_j + 1/13 T_x T_y T_z) / h^2,
  from  sum over the 3^d - 1 neighbours of u(x+d) = prod_i (2 + T_i) u - u.
* ``spectral_solve`` -- exact solve for sigma = 1 by DST-I (Dirichlet axes)
  and DCT-I (Neumann axes with node images), which diagonalise every T_i.
* ``assemble`` / ``direct_solve`` / ``cg_solve`` -- sparse matrix of the
  heterogeneous operator on the unknowns, solved by sparse LU or CG.
"""
import itertools

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

AXIS, RADIAL = 0, 1


def _faces_per_axis(dim, faces):
    faces = (faces + "DDDDDD")[:6]
    return [(faces[2 * ax], faces[2 * ax + 1]) for ax in range(dim)]


def dirichlet_mask(dim, n, faces):
    N = 2 ** n + 1
    m = np.zeros((N,) * dim, bool)
    for ax, (lo, hi) in enumerate(_faces_per_axis(dim, faces)):
        arr_ax = dim - 1 - ax  # x is the last array index
        for side, pos in ((lo, 0), (hi, N - 1)):
            if side == "D":
                sl = [slice(None)] * dim
                sl[arr_ax] = pos
                m[tuple(sl)] = True
    return m


def _second_diff(u, arr_ax, neumann_lo, neumann_hi):
    """T u along one array axis: u[j-1] - 2u[j] + u[j+1]; at a Neumann end the
    missing neighbour is the image node.  (Values at Dirichlet ends are
    irrelevant: those nodes carry no equation.)"""
    v = np.moveaxis(u, arr_ax, 0)
    out = np.empty_like(v)
    out[1:-1] = v[:-2] - 2 * v[1:-1] + v[2:]
    out[0] = (2 * v[1] - 2 * v[0]) if neumann_lo else (-2 * v[0] + v[1])
    out[-1] = (2 * v[-2] - 2 * v[-1]) if neumann_hi else (v[-2] - 2 * v[-1])
    return np.moveaxis(out, 0, arr_ax)


def kron_apply(dim, n, stencil, faces, a, u):
    """dL_1[u] for sigma = 1 at every unknown node (0 at Dirichlet nodes)."""
    h = 1.0 / 2 ** n
    fa = _faces_per_axis(dim, faces)

    def T(v, ax):
        return _second_diff(v, dim - 1 - ax, fa[ax][0] == "N", fa[ax][1] == "N")

    if stencil == AXIS:
        out = sum(T(u, ax) for ax in range(dim))
    elif dim == 2:
        out = T(u, 0) + T(u, 1) + 0.25 * T(T(u, 0), 1)
    else:
        pairs = T(T(u, 0), 1) + T(T(u, 1), 2) + T(T(u, 0), 2)
        out = (T(u, 0) + T(u, 1) + T(u, 2) + (7.0 / 26.0) * pairs
               + (1.0 / 13.0) * T(T(T(u, 0), 1), 2))
    out = out / h ** 2 + a * u
    out[dirichlet_mask(dim, n, faces)] = 0.0
    return out


def symbol_1d(N, kind):
    """Eigenvalues of T for the transform of one axis (DST-I on the N-2
    interior nodes, or DCT-I on all N nodes)."""
    if kind == "D":
        k = np.arange(1, N - 1)
    else:
        k = np.arange(N)
    # 2 cos(t) - 2 written as -4 sin^2(t/2): the difference form loses about
    # log10(1/t^2) digits on the smooth modes (1e-10 relative at N = 4097),
    # which dominate the solution
    return -4.0 * np.sin(0.5 * np.pi * k / (N - 1)) ** 2


def operator_symbol(dim, n, stencil, faces, a):
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    fa = _faces_per_axis(dim, faces)
    mus = []
    for ax in range(dim):
        lo, hi = fa[ax]
        if lo != hi:
            raise ValueError("one transform per axis needs both faces of the same kind")
        mus.append(symbol_1d(N, lo))
    grids = np.meshgrid(*mus[::-1], indexing="ij")  # array order: z, y, x
    m = grids[::-1]  # m[0] = mu_x ...
    if stencil == AXIS:
        s = sum(m)
    elif dim == 2:
        s = m[0] + m[1] + 0.25 * m[0] * m[1]
    else:
        s = (m[0] + m[1] + m[2] + (7.0 / 26.0) * (m[0] * m[1] + m[1] * m[2] + m[0] * m[2])
             + (1.0 / 13.0) * m[0] * m[1] * m[2])
    return s / h ** 2 + a


def _fwd(v, arr_ax, kind):
    if kind == "D":
        return sfft.dst(v, type=1, axis=arr_ax)
    return sfft.dct(v, type=1, axis=arr_ax)


def _inv(v, arr_ax, kind):
    if kind == "D":
        return sfft.idst(v, type=1, axis=arr_ax)
    return sfft.idct(v, type=1, axis=arr_ax)


def spectral_solve(dim, n, stencil, faces, a, f, G=None):
    """Exact solution of dL_1 u = f (sigma = 1) with Dirichlet values G; for
    pure Neumann faces with a = 0 the solution of zero trapezoid mean (f must
    then have zero trapezoid mean)."""
    N = 2 ** n + 1
    dm = dirichlet_mask(dim, n, faces)
    fa = _faces_per_axis(dim, faces)
    lift = np.zeros((N,) * dim)
    if G is not None:
        lift[dm] = np.asarray(G)[dm]
    # move the known boundary values to the right-hand side
    rhs = np.asarray(f, dtype=np.float64) - kron_apply(dim, n, stencil, faces, a, lift)
    # restrict to the transform domain of each axis (interior for Dirichlet axes)
    sl = []
    for arr_ax in range(dim):
        ax = dim - 1 - arr_ax
        sl.append(slice(1, N - 1) if fa[ax][0] == "D" else slice(None))
    sl = tuple(sl)
    v = rhs[sl].copy()
    for ax in range(dim):
        v = _fwd(v, dim - 1 - ax, fa[ax][0])
    sym = operator_symbol(dim, n, stencil, faces, a)
    if all(lo == "N" and hi == "N" for lo, hi in fa) and a == 0.0:
        # pure Neumann Poisson: the constant mode (first DCT-I coefficient, the
        # trapezoid sum) is the null space; the solution of zero mean
        sym = sym.copy()
        sym[(0,) * dim] = 1.0
        v[(0,) * dim] = 0.0
    v = v / sym
    for ax in range(dim):
        v = _inv(v, dim - 1 - ax, fa[ax][0])
    u = lift.copy()
    u[sl] = v
    return u


def _mirror(i, N):
    i = np.where(i < 0, -i, i)
    return np.where(i > N - 1, 2 * (N - 1) - i, i)


def assemble(dim, n, stencil, faces, a, sigma=None):
    """Sparse matrix of dL_1 acting on all N^d nodes (rows of Dirichlet nodes
    are empty).  Built column-block by neighbour class with numpy index
    arithmetic; Neumann faces by node images."""
    N = 2 ** n + 1
    h = 1.0 / 2 ** n
    shape = (N,) * dim
    M = N ** dim
    sig = np.ones(shape) if sigma is None else np.asarray(sigma, dtype=np.float64)
    if stencil == AXIS:
        offs = [o for o in itertools.product((-1, 0, 1), repeat=dim) if sum(map(abs, o)) == 1]
        wts = [1.0] * len(offs)
        C = 1.0
    else:
        offs = [o for o in itertools.product((-1, 0, 1), repeat=dim) if any(o)]
        wts = [1.0 / sum(x * x for x in o) for o in offs]
        C = 2.0 * dim / len(offs)
    idx = np.indices(shape)  # idx[arr_ax]
    flat = np.arange(M).reshape(shape)
    unknown = ~dirichlet_mask(dim, n, faces)
    rows, cols, vals = [], [], []
    diag = np.full(shape, float(a))
    for off, w in zip(offs, wts):
        nb = tuple(_mirror(idx[arr_ax] + off[arr_ax], N) for arr_ax in range(dim))
        coef = (C / h ** 2) * w * 0.5 * (sig[nb] + sig)
        rows.append(flat[unknown])
        cols.append(flat[nb][unknown])
        vals.append(coef[unknown])
        diag = diag - coef
    rows.append(flat[unknown])
    cols.append(flat[unknown])
    vals.append(diag[unknown])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(M, M))
    A.sum_duplicates()
    return A


def direct_solve(dim, n, stencil, faces, a, f, sigma=None, G=None):
    """Exact solution by sparse (or dense, for tiny grids) LU."""
    N = 2 ** n + 1
    shape = (N,) * dim
    A = assemble(dim, n, stencil, faces, a, sigma)
    dm = dirichlet_mask(dim, n, faces).ravel()
    un = ~dm
    ub = np.zeros(N ** dim)
    if G is not None:
        ub[dm] = np.asarray(G).ravel()[dm]
    rhs = np.asarray(f, dtype=np.float64).ravel() - A @ ub
    Auu = A[un][:, un]
    if Auu.shape[0] <= 2000:
        x = np.linalg.solve(Auu.toarray(), rhs[un])
    else:
        x = spla.spsolve(Auu.tocsc(), rhs[un])
    u = ub.copy()
    u[un] = x
    return u.reshape(shape)


def cg_solve(dim, n, stencil, a, f, sigma=None, G=None, rtol=1e-14, maxiter=20000):
    """Conjugate gradients on -A (symmetric positive definite for all-Dirichlet
    faces, sigma > 0, a <= 0)."""
    N = 2 ** n + 1
    faces = "DDDDDD"
    A = assemble(dim, n, stencil, faces, a, sigma)
    dm = dirichlet_mask(dim, n, faces).ravel()
    un = ~dm
    ub = np.zeros(N ** dim)
    if G is not None:
        ub[dm] = np.asarray(G).ravel()[dm]
    rhs = np.asarray(f, dtype=np.float64).ravel() - A @ ub
    Auu = (-A[un][:, un]).tocsr()
    d = Auu.diagonal()
    Minv = spla.LinearOperator(Auu.shape, matvec=lambda v: v / d)
    x, info = spla.cg(Auu, -rhs[un], rtol=rtol, atol=0.0, maxiter=maxiter, M=Minv)
    if info != 0:
        raise RuntimeError(f"CG did not converge (info={info})")
    u = ub.copy()
    u[un] = x
    return u.reshape((N,) * dim)
