"""FP64 CPU oracle for semi-Lagrangian Gauss-Newton-Krylov registration.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product package
``paper_1608_03630_amd`` never does, and this package imports nothing from it.

Thin ctypes wrapper over ``liboracle.so`` (built from ``oracle.c`` by
``oracle/build.py``). Every function takes and returns float64 numpy arrays in
C order ``[N1][N2][N3]`` (x3 fastest); vector fields are ``[3][N1][N2][N3]``.
What each function computes and which passage of the paper it follows is
documented beside its C implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c; the mutation tests use it to
# load deliberately broken copies in a child process.
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

MAXIT = 512


class Params(ctypes.Structure):
    """Mirror of ``oracle_params``: the solver and discretisation settings."""

    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("nt", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("beta_final", ctypes.c_double),
        ("beta_factor", ctypes.c_double),
        ("isochoric", ctypes.c_int32),
        ("forcing", ctypes.c_int32),
        ("gtol", ctypes.c_double),
        ("mismatch_tol", ctypes.c_double),
        ("max_newton", ctypes.c_int32),
        ("max_pcg", ctypes.c_int32),
        ("max_ls", ctypes.c_int32),
        ("hessian", ctypes.c_int32),
        ("armijo_c1", ctypes.c_double),
        ("gtol_level", ctypes.c_double),
        ("gnorm_ref", ctypes.c_double),
        ("gref_first", ctypes.c_double),
    ]


class Report(ctypes.Structure):
    """Mirror of ``oracle_report``."""

    _fields_ = [
        ("status", ctypes.c_int32),
        ("n_iter", ctypes.c_int32),
        ("matvecs", ctypes.c_int32),
        ("gradients", ctypes.c_int32),
        ("objectives", ctypes.c_int32),
        ("stop_reason", ctypes.c_int32),
        ("J", ctypes.c_double * MAXIT),
        ("mismatch", ctypes.c_double * MAXIT),
        ("grel", ctypes.c_double * MAXIT),
        ("alpha", ctypes.c_double * MAXIT),
        ("beta", ctypes.c_double * MAXIT),
        ("pcg_iters", ctypes.c_int32 * MAXIT),
        ("ls_trials", ctypes.c_int32 * MAXIT),
        ("final_J", ctypes.c_double),
        ("final_mismatch", ctypes.c_double),
        ("final_grel", ctypes.c_double),
        ("final_beta", ctypes.c_double),
        ("final_gref", ctypes.c_double),
        ("negative_curvature", ctypes.c_int32),
        ("descent_fallbacks", ctypes.c_int32),
    ]

    def to_dict(self):
        k = min(self.n_iter, MAXIT)
        return {
            "status": self.status,
            "n_iter": self.n_iter,
            "matvecs": self.matvecs,
            "gradients": self.gradients,
            "objectives": self.objectives,
            "stop_reason": self.stop_reason,
            "J": list(self.J[:k]),
            "mismatch": list(self.mismatch[:k]),
            "grel": list(self.grel[:k]),
            "alpha": list(self.alpha[:k]),
            "beta": list(self.beta[:k]),
            "pcg_iters": list(self.pcg_iters[:k]),
            "ls_trials": list(self.ls_trials[:k]),
            "final_J": self.final_J,
            "final_mismatch": self.final_mismatch,
            "final_grel": self.final_grel,
            "final_beta": self.final_beta,
            "final_gref": self.final_gref,
            "negative_curvature": self.negative_curvature,
            "descent_fallbacks": self.descent_fallbacks,
        }


def params(n, nt, beta, isochoric=False, beta_final=0.0, beta_factor=0.1, gtol=1e-2, mismatch_tol=0.0,
           max_newton=50, max_pcg=100, max_ls=20, forcing=0, armijo_c1=1e-4, gtol_level=0.0, gnorm_ref=0.0,
           hessian=0):
    p = Params()
    n = tuple(int(x) for x in (n if np.ndim(n) else (n, n, n)))
    p.n[:] = n
    p.nt = int(nt)
    p.beta = float(beta)
    p.beta_final = float(beta_final)
    p.beta_factor = float(beta_factor)
    p.isochoric = int(bool(isochoric))
    p.forcing = int(forcing)
    p.gtol = float(gtol)
    p.mismatch_tol = float(mismatch_tol)
    p.max_newton = int(max_newton)
    p.max_pcg = int(max_pcg)
    p.max_ls = int(max_ls)
    p.hessian = int(hessian)
    p.armijo_c1 = float(armijo_c1)
    p.gtol_level = float(gtol_level)
    p.gnorm_ref = float(gnorm_ref)
    p.gref_first = 0.0
    return p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle.build import build

        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    sig = {
        "oracle_fft3": (None, [P, P, P, I]),
        "oracle_deriv": (None, [P, I, P, P]),
        "oracle_grad": (None, [P, P, P]),
        "oracle_div": (None, [P, P, P]),
        "oracle_leray": (None, [P, P, P]),
        "oracle_even_op": (None, [P, I, I, D, P, P]),
        "oracle_precond": (None, [P, D, I, P, P]),
        "oracle_regulariser": (D, [P, D, P]),
        "oracle_resample": (None, [P, P, I, P, P]),
        "oracle_interp": (None, [P, P, P, P]),
        "oracle_interp_transpose": (None, [P, P, P, P]),
        "oracle_backtrace": (None, [P, I, P, D, P]),
        "oracle_state": (None, [P, I, P, P, P]),
        "oracle_adjoint": (None, [P, I, P, P, P, P, P]),
        "oracle_transport_forward": (I, [P, P, P, P, P]),
        "oracle_transport_adjoint": (I, [P, P, P, P]),
        "oracle_gradient": (I, [P, P, P, P, P, P, P]),
        "oracle_hessian_matvec": (I, [P, P, P, P, P]),
        "oracle_newton_matvec": (I, [P, P, P, P, P, P]),
        "oracle_objective": (I, [P, P, P, P, P, P]),
        "oracle_deformation": (I, [P, P, P, P, P, P]),
        "oracle_solve": (I, [P, P, P, P, P]),
        "oracle_num_threads": (I, []),
        "oracle_set_threads": (None, [I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _n(shape):
    return (ctypes.c_int * 3)(*[int(s) for s in shape[-3:]])


def num_threads():
    return _load().oracle_num_threads()


def set_threads(t):
    _load().oracle_set_threads(int(t))


# ---------------------------------------------------------------- spectral
def fft3(a, sign=-1):
    """Complex 3D DFT: sign -1 unnormalised forward, +1 inverse / (N1 N2 N3)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.empty_like(a)
    _load().oracle_fft3(_n(a.shape), _p(a), _p(out), int(sign))
    return out


def deriv(u, j):
    u = _f64(u)
    out = np.empty_like(u)
    _load().oracle_deriv(_n(u.shape), int(j), _p(u), _p(out))
    return out


def grad(u):
    u = _f64(u)
    out = np.empty((3,) + u.shape)
    _load().oracle_grad(_n(u.shape), _p(u), _p(out))
    return out


def div(v):
    v = _f64(v)
    out = np.empty(v.shape[1:])
    _load().oracle_div(_n(v.shape), _p(v), _p(out))
    return out


def leray(v):
    v = _f64(v)
    out = np.empty_like(v)
    _load().oracle_leray(_n(v.shape), _p(v), _p(out))
    return out


SYM_BIHARM, SYM_INVBIHARM, SYM_GAUSS, SYM_LAPLACE = 0, 1, 2, 3


def _even(u, which, par):
    u = _f64(u)
    ncomp = 1 if u.ndim == 3 else u.shape[0]
    out = np.empty_like(u)
    _load().oracle_even_op(_n(u.shape), ncomp, which, float(par), _p(u), _p(out))
    return out


def biharm(u, beta=1.0):
    """beta * lap^2 u (symbol beta |k|^4)."""
    return _even(u, SYM_BIHARM, beta)


def inv_biharm(u, beta=1.0):
    """(beta lap^2)^-1 u, identity on the mean."""
    return _even(u, SYM_INVBIHARM, beta)


def laplace(u):
    return _even(u, SYM_LAPLACE, 0.0)


def gauss(u, sigma):
    """Spectral Gaussian filter exp(-sigma^2 |k|^2 / 2), sigma in radians."""
    return _even(u, SYM_GAUSS, sigma)


def precond(r, beta, isochoric=False):
    r = _f64(r)
    out = np.empty_like(r)
    _load().oracle_precond(_n(r.shape), float(beta), int(bool(isochoric)), _p(r), _p(out))
    return out


def regulariser(v, beta):
    v = _f64(v)
    return _load().oracle_regulariser(_n(v.shape), float(beta), _p(v))


def pad(img, n):
    """Zero padding (section III-B1): the image at offset (n - m) // 2 per
    axis of an n-sized grid, zeros elsewhere."""
    img = _f64(img)
    n = tuple(int(x) for x in n)
    out = np.zeros(n)
    o = [(a - b) // 2 for a, b in zip(n, img.shape)]
    out[o[0]:o[0] + img.shape[0], o[1]:o[1] + img.shape[1], o[2]:o[2] + img.shape[2]] = img
    return out


def crop(f, m):
    """The centred m-sized block of an n-sized field (the inverse of pad)."""
    f = _f64(f)
    o = [(a - b) // 2 for a, b in zip(f.shape, m)]
    return f[o[0]:o[0] + m[0], o[1]:o[1] + m[1], o[2]:o[2] + m[2]].copy()


def resample(u, m):
    """Spectral resampling of a scalar or vector field to the grid m."""
    u = _f64(u)
    m = tuple(int(x) for x in (m if np.ndim(m) else (m, m, m)))
    ncomp = 1 if u.ndim == 3 else u.shape[0]
    out = np.empty(((ncomp,) if u.ndim == 4 else ()) + m)
    _load().oracle_resample(_n(u.shape), (ctypes.c_int * 3)(*m), ncomp, _p(u), _p(out))
    return out


# ---------------------------------------------------------- interpolation
def interp(f, D):
    """f evaluated at x_i + h*D_i by periodic tricubic Lagrange interpolation."""
    f = _f64(f)
    D = _f64(D)
    assert D.shape == (3,) + f.shape
    out = np.empty_like(f)
    _load().oracle_interp(_n(f.shape), _p(f), _p(D), _p(out))
    return out


def interp_transpose(g, D):
    g = _f64(g)
    D = _f64(D)
    out = np.empty_like(g)
    _load().oracle_interp_transpose(_n(g.shape), _p(g), _p(D), _p(out))
    return out


def backtrace(v, nt, sign=1.0):
    v = _f64(v)
    D = np.empty_like(v)
    _load().oracle_backtrace(_n(v.shape), int(nt), _p(v), float(sign), _p(D))
    return D


def state(Df, rho0, nt):
    rho0 = _f64(rho0)
    Df = _f64(Df)
    hist = np.empty((nt + 1,) + rho0.shape)
    _load().oracle_state(_n(rho0.shape), int(nt), _p(Df), _p(rho0), _p(hist))
    return hist


def adjoint(Da, lam1, nt, c=None, cX=None):
    lam1 = _f64(lam1)
    Da = _f64(Da)
    c = None if c is None else _f64(c)
    cX = None if cX is None else _f64(cX)
    hist = np.empty((nt + 1,) + lam1.shape)
    _load().oracle_adjoint(_n(lam1.shape), int(nt), _p(Da), _p(c), _p(cX), _p(lam1), _p(hist))
    return hist


def _chk(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")


def transport_forward(P, v, rho0, history=False):
    v = _f64(v)
    rho0 = _f64(rho0)
    out = np.empty_like(rho0)
    hist = np.empty((P.nt + 1,) + rho0.shape) if history else None
    _chk(_load().oracle_transport_forward(ctypes.byref(P), _p(v), _p(rho0), _p(out), _p(hist)), "transport_forward")
    return (out, hist) if history else out


def transport_adjoint(P, v, lam1):
    v = _f64(v)
    lam1 = _f64(lam1)
    out = np.empty_like(lam1)
    _chk(_load().oracle_transport_adjoint(ctypes.byref(P), _p(v), _p(lam1), _p(out)), "transport_adjoint")
    return out


def gradient(P, rhoT, rhoR, v):
    rhoT, rhoR, v = _f64(rhoT), _f64(rhoR), _f64(v)
    g = np.empty_like(v)
    J = ctypes.c_double()
    mis = ctypes.c_double()
    _chk(_load().oracle_gradient(ctypes.byref(P), _p(rhoT), _p(rhoR), _p(v), _p(g), ctypes.byref(J),
                                 ctypes.byref(mis)), "gradient")
    return g, J.value, mis.value


def hessian_matvec(P, rhoT, v, vt):
    rhoT, v, vt = _f64(rhoT), _f64(v), _f64(vt)
    out = np.empty_like(vt)
    _chk(_load().oracle_hessian_matvec(ctypes.byref(P), _p(rhoT), _p(v), _p(vt), _p(out)), "hessian_matvec")
    return out


def newton_matvec(P, rhoT, rhoR, v, vt):
    """Full Newton H(v) vt (every term of eqs. (5a)-(5e))."""
    rhoT, rhoR, v, vt = _f64(rhoT), _f64(rhoR), _f64(v), _f64(vt)
    out = np.empty_like(vt)
    _chk(_load().oracle_newton_matvec(ctypes.byref(P), _p(rhoT), _p(rhoR), _p(v), _p(vt), _p(out)), "newton_matvec")
    return out


def objective(P, rhoT, rhoR, v):
    rhoT, rhoR, v = _f64(rhoT), _f64(rhoR), _f64(v)
    J = ctypes.c_double()
    mis = ctypes.c_double()
    _chk(_load().oracle_objective(ctypes.byref(P), _p(rhoT), _p(rhoR), _p(v), ctypes.byref(J), ctypes.byref(mis)),
         "objective")
    return J.value, mis.value


def deformation(P, v):
    """Returns (u = y1 - x, det grad y1, min det, max det)."""
    v = _f64(v)
    u = np.empty_like(v)
    det = np.empty(v.shape[1:])
    mn = ctypes.c_double()
    mx = ctypes.c_double()
    _chk(_load().oracle_deformation(ctypes.byref(P), _p(v), _p(u), _p(det), ctypes.byref(mn), ctypes.byref(mx)),
         "deformation")
    return u, det, mn.value, mx.value


def solve(P, rhoT, rhoR, v0=None):
    """Gauss-Newton-Krylov solve; returns (v, report dict)."""
    rhoT, rhoR = _f64(rhoT), _f64(rhoR)
    v = np.zeros((3,) + rhoT.shape) if v0 is None else _f64(v0).copy()
    rep = Report()
    _load().oracle_solve(ctypes.byref(P), _p(rhoT), _p(rhoR), _p(v), ctypes.byref(rep))
    return v, rep.to_dict()


def coarse_params(P, m):
    """The settings of P on the grid m (every solver setting kept)."""
    q = Params()
    ctypes.memmove(ctypes.byref(q), ctypes.byref(P), ctypes.sizeof(Params))
    q.n[:] = tuple(int(x) for x in m)
    return q


def solve_grid(P, rhoT, rhoR, levels, v0=None):
    """Gauss-Newton-Krylov solve with grid continuation over `levels` grids
    (each axis halved per level; levels = 1 is solve()).

    The paper's continuation is in beta (section III-A); solving on coarser
    grids first is the other remedy for slow convergence at small beta that
    its conclusion points to. Steps, coarsest grid first:
      1. the images (and v0) are restricted to the coarse grid by spectral
         truncation (resample, section III-B1);
      2. that grid is solved by solve_grid with one level fewer, with the
         full beta continuation and the same stopping rules;
      3. its velocity is prolonged to this grid by spectral zero-padding;
      4. this grid is solved by solve() from the prolonged velocity, with the
         continuation resumed at the beta level the coarse solve ended on;
         that level keeps the gradient reference it started with on the
         coarse grid (grid L2 norms approximate the same continuous norm on
         every grid), so the grids together stop where one grid would.
    Returns (v, report of this grid's solve with a "levels" list, coarsest
    first, of the per-grid reports)."""
    rhoT, rhoR = _f64(rhoT), _f64(rhoR)
    n = tuple(int(x) for x in P.n)
    if levels <= 1:
        v, rep = solve(P, rhoT, rhoR, v0)
        rep["levels"] = [dict(rep, n=n)]
        return v, rep
    m = tuple(x // 2 for x in n)
    Pc = coarse_params(P, m)
    vc0 = None if v0 is None else resample(v0, m)
    vc, repc = solve_grid(Pc, resample(rhoT, m), resample(rhoR, m), levels - 1, vc0)
    Pf = coarse_params(P, n)
    Pf.beta = repc["final_beta"]
    Pf.gref_first = repc["final_gref"]
    v, rep = solve(Pf, rhoT, rhoR, resample(vc, n))
    rep["levels"] = repc["levels"] + [dict(rep, n=n)]
    return v, rep

