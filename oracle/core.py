"""ctypes binding of the C oracle (``sgml_oracle.c``) -- TEST INFRASTRUCTURE.

Arrays are numpy float64, C-contiguous, shaped ``(N, N)`` (index [j, i]) in
2D or ``(N, N, N)`` (index [k, j, i]) in 3D, i along x.  Faces are given as
a string of ``'D'``/``'N'`` letters in the order x-, x+, y-, y+, z-, z+.
"""
import ctypes
import os

import numpy as np

from . import build as _build

AXIS, RADIAL, RADIAL_PRINTED = 0, 1, 2
dp_t = ctypes.c_void_p
OK, E_ARG, E_DIVERGED, E_STAGNATED, E_MAXCYCLES = 0, -1, -5, -6, -7

# default pseudo-time step fractions theta (dtau = theta / D)
DEFAULT_THETA = {(AXIS, 2): 0.8, (AXIS, 3): 6.0 / 7.0, (RADIAL, 2): 1.0, (RADIAL, 3): 1.0,
                 (RADIAL_PRINTED, 2): 1.0, (RADIAL_PRINTED, 3): 1.0}


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("stencil", ctypes.c_int),
                ("face", ctypes.c_int * 6), ("a", ctypes.c_double), ("theta", ctypes.c_double),
                ("sigma", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_cycles", ctypes.c_int), ("n_r", ctypes.c_int),
                ("reading", ctypes.c_int), ("stall_window", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("norm0", ctypes.c_double),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("history", ctypes.c_double * 512), ("relax_updates", ctypes.c_longlong),
                ("restrict_updates", ctypes.c_longlong), ("interp_updates", ctypes.c_longlong),
                ("fullgrid_updates", ctypes.c_longlong)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("SGML_ORACLE_LIB")  # a planted-mistake build, for mutation checks
        if not path:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp = ctypes.c_void_p
        L.orc_apply.argtypes = [P(Problem), dp, dp]
        L.orc_apply_level.argtypes = [P(Problem), ctypes.c_int, dp, dp, dp, dp]
        L.orc_restriction.argtypes = [P(Problem), dp, dp, ctypes.c_int]
        L.orc_interp.argtypes = [P(Problem), ctypes.c_int, dp, dp]
        L.orc_relax_interp.argtypes = [P(Problem), ctypes.c_int, dp, dp, dp, dp, P(ctypes.c_double)]
        L.orc_cycle.argtypes = [P(Problem), P(Opts), dp, dp, dp, dp, dp, P(Stats)]
        L.orc_solve.argtypes = [P(Problem), P(Opts), dp, dp, dp, P(Stats)]
        L.orc_coeff_grad.argtypes = [P(Problem), dp, dp, dp]
        L.orc_adjoint.argtypes = [P(Problem), P(Opts), dp, dp, P(Stats)]
        L.orc_neumann_source.argtypes = [P(Problem), ctypes.POINTER(dp), dp, dp]
        L.orc_dirichlet_mask.argtypes = [P(Problem), dp]
        L.orc_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """A discrete problem dL(u) = f, L = div(sigma grad) + a, on [0,1]^dim."""

    def __init__(self, dim, n, stencil=AXIS, faces="DDDDDD", a=0.0, sigma=None, theta=None):
        self.dim, self.n = dim, n
        self.N = 2 ** n + 1
        self.shape = (self.N,) * dim
        self.stencil = stencil
        self.faces = faces
        self.a = float(a)
        self.theta = DEFAULT_THETA[(stencil, dim)] if theta is None else float(theta)
        self.sigma = _f64(sigma)
        if self.sigma is not None:
            assert self.sigma.shape == self.shape
        fc = (ctypes.c_int * 6)(*[0 if ch == "D" else 1 for ch in (faces + "DDDDDD")[:6]])
        self._p = Problem(dim, n, stencil, fc, self.a, self.theta, _ptr(self.sigma))

    # -- primitives -----------------------------------------------------
    def apply(self, u):
        u = _f64(u)
        out = np.empty(self.shape)
        assert lib().orc_apply(ctypes.byref(self._p), _ptr(u), _ptr(out)) == OK
        return out

    def apply_level(self, nu, u, sig_nu=None, with_diag=False):
        u = _f64(u)
        sig_nu = _f64(sig_nu)
        out = np.empty(self.shape)
        diag = np.empty(self.shape) if with_diag else None
        assert lib().orc_apply_level(ctypes.byref(self._p), nu, _ptr(sig_nu), _ptr(u), _ptr(out),
                                     _ptr(diag)) == OK
        return (out, diag) if with_diag else out

    def restriction(self, f, nu):
        f = _f64(f)
        out = np.empty(self.shape)
        assert lib().orc_restriction(ctypes.byref(self._p), _ptr(f), _ptr(out), nu) == OK
        return out

    def interp(self, nu, delta):
        delta = _f64(delta)
        out = np.empty(self.shape)
        assert lib().orc_interp(ctypes.byref(self._p), nu, _ptr(delta), _ptr(out)) == OK
        return out

    def relax_interp(self, nu, u, g_nu, sig_nu=None, G=None):
        u = _f64(u).copy()
        g_nu, sig_nu, G = _f64(g_nu), _f64(sig_nu), _f64(G)
        pres = ctypes.c_double(0.0)
        assert lib().orc_relax_interp(ctypes.byref(self._p), nu, _ptr(u), _ptr(g_nu), _ptr(sig_nu),
                                      _ptr(G), ctypes.byref(pres)) == OK
        return u, pres.value

    def dirichlet_mask(self):
        m = np.empty(self.shape, dtype=np.uint8)
        assert lib().orc_dirichlet_mask(ctypes.byref(self._p), _ptr(m)) == OK
        return m.astype(bool)

    # -- cycle / solve --------------------------------------------------
    @staticmethod
    def _opts(tol=1e-12, max_cycles=100, n_r=2, reading=0, stall_window=0):
        return Opts(tol, max_cycles, n_r, reading, stall_window)

    def cycle(self, src, G=None, n_r=2, reading=0, with_pres=False, with_trace=False):
        """One cycle from zero.  Returns e, plus the per-visit pseudo-residuals
        and/or the per-visit states of e when asked."""
        src, G = _f64(src), _f64(G)
        e = np.empty(self.shape)
        nvis = len(schedule(self.n, n_r, reading))
        pres = np.zeros(nvis)
        trace = np.zeros((nvis,) + self.shape) if with_trace else None
        st = Stats()
        o = self._opts(n_r=n_r, reading=reading)
        assert lib().orc_cycle(ctypes.byref(self._p), ctypes.byref(o), _ptr(src), _ptr(G), _ptr(e),
                               _ptr(pres), _ptr(trace), ctypes.byref(st)) == OK
        out = (e,)
        if with_pres:
            out += (pres,)
        if with_trace:
            out += (trace,)
        return out if len(out) > 1 else e

    def solve(self, f, G=None, tol=1e-12, max_cycles=100, n_r=2, reading=0, stall_window=0):
        """Returns (u, info) with info a dict of the solve statistics."""
        f, G = _f64(f), _f64(G)
        u = np.empty(self.shape)
        st = Stats()
        o = self._opts(tol, max_cycles, n_r, reading, stall_window)
        rc = lib().orc_solve(ctypes.byref(self._p), ctypes.byref(o), _ptr(f), _ptr(G), _ptr(u),
                             ctypes.byref(st))
        assert rc != E_ARG
        info = dict(status=st.status, cycles=st.cycles, norm0=st.norm0, relres=st.relres,
                    relres_true=st.relres_true, history=list(st.history[:min(st.cycles, 512)]),
                    relax_updates=st.relax_updates, restrict_updates=st.restrict_updates,
                    interp_updates=st.interp_updates, fullgrid_updates=st.fullgrid_updates)
        return u, info

    def adjoint(self, g, tol=1e-12, max_cycles=100, n_r=2, reading=0, stall_window=0):
        """Solve dL^T lam = g (lam = 0 on Dirichlet nodes); returns (lam, info)."""
        g = _f64(g)
        lam = np.empty(self.shape)
        st = Stats()
        o = self._opts(tol, max_cycles, n_r, reading, stall_window)
        rc = lib().orc_adjoint(ctypes.byref(self._p), ctypes.byref(o), _ptr(g), _ptr(lam), ctypes.byref(st))
        assert rc != E_ARG
        return lam, dict(status=st.status, cycles=st.cycles, relres=st.relres)

    def neumann_source(self, f, flux):
        """f minus the Neumann-data part of dL_1: flux is a sequence of 2*dim
        face arrays (outward normal derivative, shape (N,)*(dim-1), or None)."""
        f = _f64(f)
        keep = [None if g is None else _f64(g) for g in (list(flux) + [None] * 6)[:6]]
        arr = (dp_t * 6)(*[None if g is None else g.ctypes.data for g in keep])
        out = np.empty(self.shape)
        assert lib().orc_neumann_source(ctypes.byref(self._p), arr, _ptr(f), _ptr(out)) == OK
        return out

    def coeff_grad(self, u, lam):
        u, lam = _f64(u), _f64(lam)
        out = np.empty(self.shape)
        assert lib().orc_coeff_grad(ctypes.byref(self._p), _ptr(u), _ptr(lam), _ptr(out)) == OK
        return out


def threads():
    """Number of host threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def schedule(n, n_r=2, reading=0):
    cap = 8 * n + 16
    lev = np.zeros(cap, dtype=np.int32)
    cnt = np.zeros(cap, dtype=np.int32)
    ln = lib().orc_schedule(n, n_r, reading, _ptr(lev), _ptr(cnt), cap)
    return list(zip(lev[:ln].tolist(), cnt[:ln].tolist()))
