"""Thin ctypes binding of ``libsgml.so`` (C-ABI: include/sgml.h).

Argument marshalling only: every step of the solve runs in the HIP
library.  torch tensors serve as device buffers (their ``data_ptr``) and
torch's current stream as the HIP stream.  If the library is missing this
module raises on first use -- there is no fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgml.so")

OK, E_ARG, E_SHAPE, E_WORKSPACE, E_HIP = 0, -1, -2, -3, -4
E_DIVERGED, E_STAGNATED, E_MAXCYCLES, E_UNSUPPORTED = -5, -6, -7, -8
DIRICHLET, NEUMANN = 0, 1
AXIS, RADIAL = 0, 1
FP64, MIXED = 0, 1
SCHEDULE_ONCE, SCHEDULE_EACH = 0, 1
HIST = 512
MAX_VISITS = 128
PROF_CLASSES = 5
PROF_NAMES = ("sweep0", "visit0_inject", "visit0", "cycle_end", "visit0_end")


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("stencil", ctypes.c_int),
                ("face", ctypes.c_int * 6), ("a", ctypes.c_double), ("theta", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_cycles", ctypes.c_int), ("n_r", ctypes.c_int),
                ("schedule", ctypes.c_int), ("precision", ctypes.c_int),
                ("record_pres", ctypes.c_int), ("profile", ctypes.c_int),
                ("coarse_nodes", ctypes.c_int), ("stall_window", ctypes.c_int),
                ("fuse", ctypes.c_int), ("chunk_rows", ctypes.c_int), ("z_chunk", ctypes.c_int),
                ("graphs", ctypes.c_int), ("fuse_end", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("norm0", ctypes.c_double),
                ("relres", ctypes.c_double), ("history", ctypes.c_double * HIST),
                ("visits", ctypes.c_int), ("pres", ctypes.c_double * MAX_VISITS),
                ("node_updates", ctypes.c_longlong), ("ms", ctypes.c_float),
                ("prof_launches", ctypes.c_int * PROF_CLASSES),
                ("prof_ms", ctypes.c_float * PROF_CLASSES),
                ("prof_sweeps", ctypes.c_int * PROF_CLASSES), ("prof_untimed", ctypes.c_int)]

    def as_dict(self):
        return dict(status=self.status, cycles=self.cycles, norm0=self.norm0, relres=self.relres,
                    history=list(self.history[:min(self.cycles, HIST)]),
                    pres=list(self.pres[:self.visits]), node_updates=self.node_updates,
                    ms=self.ms,
                    prof={PROF_NAMES[c]: dict(launches=self.prof_launches[c], ms=self.prof_ms[c],
                                              sweeps=self.prof_sweeps[c])
                          for c in range(PROF_CLASSES)},
                    prof_untimed=self.prof_untimed)


class SGMLError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1703_07206_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        L.sgml_workspace_bytes.restype = ctypes.c_size_t
        L.sgml_workspace_bytes.argtypes = [P(Problem), ctypes.c_int]
        L.sgml_plan_create.argtypes = [P(Problem), ctypes.c_int, vp, ctypes.c_size_t, P(vp)]
        L.sgml_plan_set_coeffs.argtypes = [vp, vp, vp]
        L.sgml_solve.argtypes = [vp, vp, vp, vp, P(Opts), vp, P(Stats)]
        L.sgml_solve_noalloc.argtypes = [vp, vp, vp, vp, P(Opts), vp, P(Stats)]
        L.sgml_workspace_bytes_batch.restype = ctypes.c_size_t
        L.sgml_workspace_bytes_batch.argtypes = [P(Problem), ctypes.c_int, ctypes.c_int]
        L.sgml_plan_create_batch.argtypes = [P(Problem), ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, P(vp)]
        L.sgml_solve_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, P(Opts), vp, vp]
        L.sgml_residual.argtypes = [vp, vp, vp, vp, vp, P(ctypes.c_double), P(ctypes.c_double), vp]
        L.sgml_adjoint.argtypes = [vp, vp, vp, P(Opts), vp, P(Stats)]
        L.sgml_coeff_grad.argtypes = [vp, vp, vp, vp, vp]
        L.sgml_neumann_source.argtypes = [vp, vp, vp, vp, vp]
        L.sgml_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int,
                                    P(ctypes.c_int)]
        L.sgml_status_string.restype = ctypes.c_char_p
        L.sgml_status_string.argtypes = [ctypes.c_int]
        L.sgml_plan_destroy.argtypes = [vp]
        L.sgml_plan_destroy.restype = None
        for name in ("sgml_plan_create", "sgml_plan_set_coeffs", "sgml_solve", "sgml_solve_noalloc", "sgml_plan_create_batch", "sgml_solve_batch",
                     "sgml_residual",
                     "sgml_adjoint", "sgml_coeff_grad", "sgml_neumann_source", "sgml_schedule"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status):
    return lib().sgml_status_string(int(status)).decode()


def _faces(dim, faces):
    faces = (faces + "DDDDDD")[:6]
    return (ctypes.c_int * 6)(*[DIRICHLET if c == "D" else NEUMANN for c in faces])


def make_problem(dim, n, stencil=AXIS, faces="DDDDDD", a=0.0, theta=0.0):
    return Problem(dim, n, stencil, _faces(dim, faces), float(a), float(theta))


def workspace_bytes(dim, n, stencil=AXIS, faces="DDDDDD", a=0.0, precision=FP64):
    return lib().sgml_workspace_bytes(ctypes.byref(make_problem(dim, n, stencil, faces, a)), precision)


def schedule(n, n_r=2, sched=SCHEDULE_ONCE):
    cap = 8 * n + 16
    lev = (ctypes.c_int * cap)()
    cnt = (ctypes.c_int * cap)()
    ln = ctypes.c_int(0)
    rc = lib().sgml_schedule(n, n_r, sched, ctypes.addressof(lev), ctypes.addressof(cnt), cap,
                             ctypes.byref(ln))
    if rc != OK:
        raise SGMLError(rc, "sgml_schedule")
    return [(lev[i], cnt[i]) for i in range(ln.value)]


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Plan:
    """A solver plan: problem description, device workspace and coefficients.

    Parameters mirror ``sgml_problem``: ``dim`` 2 or 3, ``n`` with
    N = 2^n + 1, ``stencil`` AXIS or RADIAL, ``faces`` a string of 'D'/'N'
    for x-, x+, y-, y+, z-, z+, ``a`` the constant of L = div(sigma grad) + a,
    ``sigma`` an optional (N,)*dim float64 CUDA tensor, ``precision`` the
    highest precision mode the plan will be asked for (MIXED covers both).
    ``workspace=False`` creates a plan without a device workspace, which only
    ``solve_noalloc`` (and ``coeff_grad``) can use.  ``nrhs > 1`` creates a
    batch plan for ``solve_batch`` (one workspace slice and stream per
    right-hand side, one coefficient pyramid).
    """

    def __init__(self, dim, n, stencil=AXIS, faces="DDDDDD", a=0.0, sigma=None, precision=FP64,
                 theta=0.0, device=None, workspace=True, nrhs=1):
        L = lib()
        self.dim, self.n = dim, n
        self.N = 2 ** n + 1
        self.shape = (self.N,) * dim
        self.stencil, self.faces, self.a = stencil, faces, float(a)
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._prob = make_problem(dim, n, stencil, faces, a, theta)
        self.nrhs = int(nrhs)
        if self.nrhs > 1:
            nbytes = L.sgml_workspace_bytes_batch(ctypes.byref(self._prob), precision, self.nrhs)
        else:
            nbytes = L.sgml_workspace_bytes(ctypes.byref(self._prob), precision)
        if nbytes == 0:
            raise SGMLError(E_ARG, "sgml_workspace_bytes")
        self.workspace_bytes = nbytes
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device) if workspace else None
            h = ctypes.c_void_p()
            if self.nrhs > 1:
                rc = L.sgml_plan_create_batch(ctypes.byref(self._prob), precision, self.nrhs,
                                              self.workspace.data_ptr(), nbytes, ctypes.byref(h))
            else:
                rc = L.sgml_plan_create(ctypes.byref(self._prob), precision,
                                        self.workspace.data_ptr() if workspace else None,
                                        nbytes if workspace else 0, ctypes.byref(h))
        if rc != OK:
            raise SGMLError(rc, "sgml_plan_create")
        self._h = h
        self.sigma = None
        self.set_coeffs(sigma)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.sgml_plan_destroy(h)
            self._h = None

    def _check(self, t, name):
        if t is not None and tuple(t.shape) != self.shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.shape}")

    def set_coeffs(self, sigma, stream=None):
        self._check(sigma, "sigma")
        self.sigma = sigma  # the plan borrows it: keep a reference
        rc = lib().sgml_plan_set_coeffs(self._h, _ptr(sigma), _stream(stream))
        if rc != OK:
            raise SGMLError(rc, "sgml_plan_set_coeffs")

    def opts(self, tol=1e-12, max_cycles=100, n_r=2, schedule=SCHEDULE_ONCE, precision=None,
             record_pres=False, profile=False, coarse_nodes=0, stall_window=0, fuse=0, chunk_rows=0,
             z_chunk=0, graphs=0, fuse_end=0):
        return Opts(tol, max_cycles, n_r, schedule, self.precision if precision is None else precision,
                    int(record_pres), int(profile), int(coarse_nodes), int(stall_window), int(fuse),
                    int(chunk_rows), int(z_chunk), int(graphs), int(fuse_end))

    def solve(self, f, G=None, u=None, raise_on_failure=True, stream=None, **kw):
        """Solve dL(u) = f; returns (u, stats dict)."""
        self._check(f, "f")
        self._check(G, "G")
        if u is None:
            u = torch.empty_like(f)
        o = self.opts(**kw)
        st = Stats()
        rc = lib().sgml_solve(self._h, _ptr(f), _ptr(G), _ptr(u), ctypes.byref(o), _stream(stream),
                              ctypes.byref(st))
        if rc in (E_ARG, E_SHAPE, E_WORKSPACE, E_HIP, E_UNSUPPORTED) or (rc != OK and raise_on_failure):
            raise SGMLError(rc, "sgml_solve")
        return u, st.as_dict()

    def solve_batch(self, F, G=None, U=None, raise_on_failure=True, stream=None, **kw):
        """Solve dL(u_r) = f_r for the right-hand sides F[0..k-1] (shape
        (k,) + grid shape) at once; G: (k,) + grid shape or None.  Returns
        (U, list of k stats dicts)."""
        k = F.shape[0]
        if tuple(F.shape[1:]) != self.shape or (G is not None and tuple(G.shape) != tuple(F.shape)):
            raise ValueError("F (and G) must have shape (k,) + the grid shape")
        if U is None:
            U = torch.empty_like(F)
        o = self.opts(**kw)
        st = (Stats * k)()
        rc = lib().sgml_solve_batch(self._h, k, _ptr(F), _ptr(G), _ptr(U), ctypes.byref(o), _stream(stream),
                                    ctypes.addressof(st))
        if rc in (E_ARG, E_SHAPE, E_WORKSPACE, E_HIP, E_UNSUPPORTED) or (rc != OK and raise_on_failure):
            raise SGMLError(rc, "sgml_solve_batch")
        return U, [st[r].as_dict() for r in range(k)]

    def solve_noalloc(self, f, G=None, u=None, raise_on_failure=True, stream=None, **kw):
        """``solve`` through sgml_solve_noalloc: the library's static per-device
        workspace instead of the plan's; ``u`` should be given by callers that
        cannot allocate (else it is allocated here, by torch)."""
        self._check(f, "f")
        self._check(G, "G")
        if u is None:
            u = torch.empty_like(f)
        o = self.opts(**kw)
        st = Stats()
        rc = lib().sgml_solve_noalloc(self._h, _ptr(f), _ptr(G), _ptr(u), ctypes.byref(o), _stream(stream),
                                      ctypes.byref(st))
        if rc in (E_ARG, E_SHAPE, E_WORKSPACE, E_HIP, E_UNSUPPORTED) or (rc != OK and raise_on_failure):
            raise SGMLError(rc, "sgml_solve_noalloc")
        return u, st.as_dict()

    def residual(self, f, u, G=None, r=None, stream=None):
        """Returns (r or None, max|r|, norm0)."""
        rmax, norm0 = ctypes.c_double(), ctypes.c_double()
        rc = lib().sgml_residual(self._h, _ptr(f), _ptr(G), _ptr(u), _ptr(r), ctypes.byref(rmax),
                                 ctypes.byref(norm0), _stream(stream))
        if rc != OK:
            raise SGMLError(rc, "sgml_residual")
        return r, rmax.value, norm0.value

    def adjoint(self, g, lam=None, raise_on_failure=True, stream=None, **kw):
        if lam is None:
            lam = torch.empty_like(g)
        o = self.opts(**kw)
        st = Stats()
        rc = lib().sgml_adjoint(self._h, _ptr(g), _ptr(lam), ctypes.byref(o), _stream(stream),
                                ctypes.byref(st))
        if rc in (E_ARG, E_SHAPE, E_WORKSPACE, E_HIP, E_UNSUPPORTED) or (rc != OK and raise_on_failure):
            raise SGMLError(rc, "sgml_adjoint")
        return lam, st.as_dict()

    def neumann_source(self, f, flux, out=None, stream=None):
        """f minus the Neumann-data part of dL (sgml_neumann_source): flux is a
        sequence of up to 6 face tensors (outward normal derivative, shape
        (N,)*(dim-1), float64 on the device) or None."""
        if out is None:
            out = torch.empty_like(f)
        faces = list(flux) + [None] * (6 - len(flux))
        for g in faces:
            if g is not None and tuple(g.shape) != (self.N,) * (self.dim - 1):
                raise ValueError(f"face data of shape {tuple(g.shape)}, expected {(self.N,) * (self.dim - 1)}")
        arr = (ctypes.c_void_p * 6)(*[_ptr(g) for g in faces])
        rc = lib().sgml_neumann_source(self._h, _ptr(f), ctypes.addressof(arr), _ptr(out), _stream(stream))
        if rc != OK:
            raise SGMLError(rc, "sgml_neumann_source")
        return out

    def coeff_grad(self, u, lam, grad=None, stream=None):
        if grad is None:
            grad = torch.empty_like(u)
        rc = lib().sgml_coeff_grad(self._h, _ptr(u), _ptr(lam), _ptr(grad), _stream(stream))
        if rc != OK:
            raise SGMLError(rc, "sgml_coeff_grad")
        return grad


def solve(f, sigma=None, a=0.0, G=None, faces="DDDDDD", stencil=AXIS, tol=1e-12, precision=FP64,
          **kw):
    """One-shot solve of div(sigma grad u) + a u = f on the grid of f."""
    dim = f.dim()
    n = (f.shape[0] - 1).bit_length() - 1
    plan = Plan(dim, n, stencil, faces, a, sigma, precision)
    return plan.solve(f, G, tol=tol, precision=precision, **kw)
