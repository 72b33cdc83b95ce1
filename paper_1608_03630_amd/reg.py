"""Python binding of libreg (include/reg.h): argument marshalling only.

Every function here has the name of the C entry point it calls and passes
torch tensors' device pointers and the current HIP stream through ctypes; all
arithmetic runs in the library's HIP kernels. Host-side checks cover what the C
side cannot see: tensor dtype, device, contiguity and element count.

The library must be built (``__graft_entry__.build()`` or
``python paper_1608_03630_amd/build.py``); importing a function that needs it
raises if ``libreg.so`` is missing. There is no fallback path.
"""
import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreg.so")
REG_MAXIT = 512
REG_MAXLEVELS = 4

STATUS = {
    0: "REG_OK", 1: "REG_EINVAL", 2: "REG_ENOMEM", 3: "REG_EHIP", 4: "REG_ENONFINITE",
    6: "REG_ELINESEARCH", 7: "REG_ENONDIFFEO", 8: "REG_ENOTIMPL",
}
REG_OK, REG_EINVAL, REG_ENOMEM, REG_EHIP, REG_ENONFINITE = 0, 1, 2, 3, 4
REG_ELINESEARCH, REG_ENONDIFFEO = 6, 7

SPEC_BIHARM, SPEC_INVBIHARM, SPEC_GAUSS, SPEC_LERAY = 0, 1, 2, 3


class RegError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class reg_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("nt", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("beta_final", ctypes.c_double),
        ("beta_factor", ctypes.c_double),
        ("isochoric", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("gtol", ctypes.c_double),
        ("mismatch_tol", ctypes.c_double),
        ("max_newton", ctypes.c_int32),
        ("max_pcg", ctypes.c_int32),
        ("max_ls", ctypes.c_int32),
        ("forcing", ctypes.c_int32),
        ("armijo_c1", ctypes.c_double),
        ("gnorm_ref", ctypes.c_double),
        ("gtol_level", ctypes.c_double),
        ("grid_levels", ctypes.c_int32),
        ("hessian", ctypes.c_int32),
        ("det_check", ctypes.c_int32),
        ("recompute_grad_rho", ctypes.c_int32),
    ]


class reg_report(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("n_iter", ctypes.c_int32),
        ("matvecs", ctypes.c_int32),
        ("gradients", ctypes.c_int32),
        ("objectives", ctypes.c_int32),
        ("stop_reason", ctypes.c_int32),
        ("J", ctypes.c_double * REG_MAXIT),
        ("mismatch", ctypes.c_double * REG_MAXIT),
        ("grel", ctypes.c_double * REG_MAXIT),
        ("alpha", ctypes.c_double * REG_MAXIT),
        ("beta", ctypes.c_double * REG_MAXIT),
        ("pcg_iters", ctypes.c_int32 * REG_MAXIT),
        ("ls_trials", ctypes.c_int32 * REG_MAXIT),
        ("final_J", ctypes.c_double),
        ("final_mismatch", ctypes.c_double),
        ("final_grel", ctypes.c_double),
        ("seconds_total", ctypes.c_double),
        ("seconds_matvec", ctypes.c_double),
        ("seconds_gradient", ctypes.c_double),
        ("seconds_objective", ctypes.c_double),
        ("seconds_precond", ctypes.c_double),
        ("interps", ctypes.c_int64),
        ("final_beta", ctypes.c_double),
        ("final_gref", ctypes.c_double),
        ("grid_levels", ctypes.c_int32),
        ("level_n", (ctypes.c_int32 * 3) * REG_MAXLEVELS),
        ("level_iters", ctypes.c_int32 * REG_MAXLEVELS),
        ("level_matvecs", ctypes.c_int32 * REG_MAXLEVELS),
        ("level_seconds", ctypes.c_double * REG_MAXLEVELS),
        ("level_mismatch", ctypes.c_double * REG_MAXLEVELS),
        ("level_beta", ctypes.c_double * REG_MAXLEVELS),
        ("negative_curvature", ctypes.c_int32),
        ("descent_fallbacks", ctypes.c_int32),
        ("fft3d", ctypes.c_int64),
        ("fft_lines", ctypes.c_int64),
        ("det_min", ctypes.c_double),
        ("det_max", ctypes.c_double),
        ("alg_bytes", ctypes.c_double),
    ]

    def to_dict(self):
        k = min(self.n_iter, REG_MAXIT)
        out = {f: getattr(self, f) for f in ("status", "n_iter", "matvecs", "gradients", "objectives",
                                             "stop_reason", "final_J", "final_mismatch", "final_grel",
                                             "seconds_total", "seconds_matvec", "seconds_gradient",
                                             "seconds_objective", "seconds_precond", "interps", "final_beta",
                                             "final_gref", "negative_curvature", "descent_fallbacks", "fft3d",
                                             "fft_lines", "det_min", "det_max", "alg_bytes")}
        for f in ("J", "mismatch", "grel", "alpha", "beta", "pcg_iters", "ls_trials"):
            out[f] = list(getattr(self, f)[:k])
        out["levels"] = [{"n": tuple(self.level_n[i]), "n_iter": self.level_iters[i],
                          "matvecs": self.level_matvecs[i], "seconds": self.level_seconds[i],
                          "final_mismatch": self.level_mismatch[i], "final_beta": self.level_beta[i]}
                         for i in range(min(self.grid_levels, REG_MAXLEVELS))]
        return out


_lib = None
_P = ctypes.c_void_p
# reg_log_fn: void (*)(const char *json, void *user)
LOG_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_void_p)

_SIGS = {
    "reg_set_log": [_P, LOG_FN, _P],
    "reg_default_params": [ctypes.POINTER(reg_params)],
    "reg_workspace_size": [ctypes.POINTER(reg_params), ctypes.POINTER(ctypes.c_size_t)],
    "reg_create": [ctypes.POINTER(reg_params), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "reg_destroy": [_P],
    "reg_set_beta": [_P, ctypes.c_double],
    "reg_set_solver": [_P, ctypes.POINTER(reg_params)],
    "reg_set_images": [_P, _P, _P],
    "reg_interp": [_P, _P, _P, _P],
    "reg_pad": [_P, ctypes.POINTER(ctypes.c_int32), _P, _P],
    "reg_crop": [_P, ctypes.POINTER(ctypes.c_int32), _P, _P],
    "reg_interp_noalloc": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P],
    "reg_backtrace": [_P, _P, ctypes.c_double, _P],
    "reg_deriv": [_P, ctypes.c_int, _P, _P],
    "reg_grad": [_P, _P, _P],
    "reg_div": [_P, _P, _P],
    "reg_spectral": [_P, ctypes.c_int, ctypes.c_double, ctypes.c_int, _P, _P],
    "reg_precond": [_P, _P, _P],
    "reg_transport_forward": [_P, _P, _P, _P],
    "reg_transport_adjoint": [_P, _P, _P, _P],
    "reg_gradient": [_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                     ctypes.POINTER(ctypes.c_double)],
    "reg_objective": [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "reg_hessian_matvec": [_P, _P, _P],
    "reg_solve": [_P, _P, ctypes.POINTER(reg_report)],
    "reg_deformation": [_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "reg_dot": [_P, ctypes.c_int, _P, _P, ctypes.POINTER(ctypes.c_double)],
    "reg_resample": [_P, _P, ctypes.c_int, _P, _P],
    "reg_profile": [_P, ctypes.c_int],
    "reg_profile_read": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "reg_batch_workspace_size": [ctypes.POINTER(reg_params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "reg_batch_create": [ctypes.POINTER(reg_params), ctypes.c_int32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "reg_batch_destroy": [_P],
    "reg_batch_ctx": [_P, ctypes.c_int32, ctypes.POINTER(_P)],
    "reg_batch_set_launch": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "reg_batch_set_tile": [_P, ctypes.c_int32, ctypes.c_int32],
    "reg_batch_launch_info": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
    "reg_batch_stats": [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_int64)],
    "reg_batch_profile": [_P, ctypes.c_int],
    "reg_batch_profile_read": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "reg_batch_transport_forward": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)],
    "reg_batch_gradient": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "reg_batch_hessian_matvec": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)],
    "reg_batch_solve": [_P, ctypes.POINTER(_P), ctypes.POINTER(reg_report)],
    "reg_net_param_count": [ctypes.POINTER(ctypes.c_int64)],
    "reg_net_workspace_size": [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "reg_net_create": [ctypes.c_int32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "reg_net_destroy": [_P],
    "reg_net_set_params": [_P, _P],
    "reg_net_get_params": [_P, _P],
    "reg_net_forward": [_P, _P, _P, _P],
    "reg_net_activation": [_P, ctypes.c_int32, _P],
    "reg_net_loss_grad": [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)],
    "reg_net_backward": [_P, _P, _P],
    "reg_net_step": [_P, _P, ctypes.c_double],
    "reg_net_train_step": [_P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                           ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
    "reg_warmstart": [_P, _P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
}

KERNEL_KINDS = ["interp", "backtrace", "adjoint", "incstate", "deform", "deriv", "fft3d", "symbol", "reduce",
                "vector", "graph"]


def lib():
    """Loads libreg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.reg_last_error.argtypes = [_P]
        L.reg_last_error.restype = ctypes.c_char_p
        L.reg_batch_last_error.argtypes = [_P]
        L.reg_batch_last_error.restype = ctypes.c_char_p
        L.reg_net_last_error.argtypes = [_P]
        L.reg_net_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _chk(st, ctx=None, what=""):
    if st != REG_OK:
        msg = lib().reg_last_error(ctx).decode() if ctx else ""
        raise RegError(st, f"{what}: {msg}")


def reg_default_params(n=(64, 64, 64), **kw):
    p = reg_params()
    _chk(lib().reg_default_params(ctypes.byref(p)), what="reg_default_params")
    n = tuple(int(x) for x in (n if hasattr(n, "__len__") else (n, n, n)))
    p.n[:] = n
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, type(getattr(p, k))(v))
    return p


def reg_workspace_size(p):
    b = ctypes.c_size_t()
    _chk(lib().reg_workspace_size(ctypes.byref(p), ctypes.byref(b)), what="reg_workspace_size")
    return b.value


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def reg_interp_noalloc(f, D, out, stream=None):
    """reg_interp without a context (the entry point that allocates nothing):
    f and out are [n0][n1][n2] float32 or float64 CUDA tensors, D is [3][n0][n1][n2]
    of the same dtype; out is written in place."""
    for t, name in ((f, "f"), (D, "D"), (out, "out")):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor")
        if t.dtype != f.dtype or f.dtype not in (torch.float32, torch.float64):
            raise TypeError(f"{name} must be float32 or float64 like f")
    if f.dim() != 3 or tuple(out.shape) != tuple(f.shape) or tuple(D.shape) != (3,) + tuple(f.shape):
        raise ValueError("f, out must be [n0][n1][n2] and D [3][n0][n1][n2]")
    n = (ctypes.c_int32 * 3)(*f.shape)
    _chk(lib().reg_interp_noalloc(int(f.dtype == torch.float64), n, ctypes.c_void_p(f.data_ptr()),
                                  ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
         what="reg_interp_noalloc")
    return out


class Context:
    """One reg_ctx over a torch-allocated workspace, bound to one stream (or,
    with `borrowed`, a view of a context that a Batch owns)."""

    def __init__(self, params, device="cuda", stream=None, borrowed=None):
        self.params = params
        self.device = torch.device(device)
        self.dtype = torch.float64 if params.prec else torch.float32  # image-space fields
        self.vdtype = torch.float64  # velocity-space vectors
        self.shape = tuple(params.n)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.owned = borrowed is None
        if borrowed is not None:
            self.workspace = None
            self.stream = None
            self.handle = borrowed
            return
        nbytes = reg_workspace_size(params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _chk(lib().reg_create(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                              _stream_ptr(stream), ctypes.byref(h)), what="reg_create")
        self.handle = h

    def close(self):
        if self.handle and self.owned:
            lib().reg_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ checks
    def _t(self, t, ncomp, name, vel=False):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must live on the GPU")
        want = self.vdtype if vel else self.dtype
        if t.dtype != want:
            raise TypeError(f"{name} must be {want}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != ncomp * self.N:
            raise ValueError(f"{name} must hold {ncomp} x {self.shape} elements, got shape {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, ncomp=1, vel=False):
        shape = self.shape if ncomp == 1 else (ncomp,) + self.shape
        return torch.empty(shape, dtype=self.vdtype if vel else self.dtype, device=self.device)

    # ------------------------------------------------------ entry points
    def reg_set_beta(self, beta):
        _chk(lib().reg_set_beta(self.handle, float(beta)), self.handle, "reg_set_beta")

    def reg_set_log(self, fn=None):
        """fn(dict) after every accepted Newton step of reg_solve (None: off)."""
        if fn is None:
            self._log_cb = None
            _chk(lib().reg_set_log(self.handle, LOG_FN(), None), self.handle, "reg_set_log")
            return
        self._log_cb = LOG_FN(lambda line, user: fn(json.loads(line.decode())))
        _chk(lib().reg_set_log(self.handle, self._log_cb, None), self.handle, "reg_set_log")

    def reg_set_solver(self, params):
        _chk(lib().reg_set_solver(self.handle, ctypes.byref(params)), self.handle, "reg_set_solver")
        self.params = params

    def reg_set_images(self, rho_T, rho_R):
        _chk(lib().reg_set_images(self.handle, self._t(rho_T, 1, "rho_T"), self._t(rho_R, 1, "rho_R")),
             self.handle, "reg_set_images")

    def reg_interp(self, f, D, out=None):
        out = self.empty(1) if out is None else out
        _chk(lib().reg_interp(self.handle, self._t(f, 1, "f"), self._t(D, 3, "D"), self._t(out, 1, "out")),
             self.handle, "reg_interp")
        return out

    def reg_backtrace(self, v, sign=1.0, D=None):
        D = self.empty(3) if D is None else D
        _chk(lib().reg_backtrace(self.handle, self._t(v, 3, "v", True), float(sign), self._t(D, 3, "D")), self.handle,
             "reg_backtrace")
        return D

    def reg_deriv(self, axis, u, out=None):
        out = self.empty(1) if out is None else out
        _chk(lib().reg_deriv(self.handle, int(axis), self._t(u, 1, "u"), self._t(out, 1, "out")), self.handle,
             "reg_deriv")
        return out

    def reg_grad(self, u, out=None):
        out = self.empty(3) if out is None else out
        _chk(lib().reg_grad(self.handle, self._t(u, 1, "u"), self._t(out, 3, "out")), self.handle, "reg_grad")
        return out

    def reg_div(self, v, out=None):
        out = self.empty(1) if out is None else out
        _chk(lib().reg_div(self.handle, self._t(v, 3, "v"), self._t(out, 1, "out")), self.handle, "reg_div")
        return out

    def reg_spectral(self, op, scale, v, out=None):
        ncomp = 1 if v.dim() == 3 else v.shape[0]
        out = self.empty(ncomp) if out is None else out
        _chk(lib().reg_spectral(self.handle, int(op), float(scale), ncomp, self._t(v, ncomp, "v"),
                                self._t(out, ncomp, "out")), self.handle, "reg_spectral")
        return out

    def reg_resample(self, dst, x, out=None):
        """Spectral resampling of x (this context's grid) onto dst's grid."""
        ncomp = 1 if x.dim() == 3 else x.shape[0]
        out = dst.empty(ncomp) if out is None else out
        _chk(lib().reg_resample(self.handle, dst.handle, ncomp, self._t(x, ncomp, "x"), dst._t(out, ncomp, "out")),
             self.handle, "reg_resample")
        return out

    def _m(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous() or t.dtype != self.dtype:
            raise TypeError(f"{name} must be a contiguous {self.dtype} CUDA tensor")
        if t.dim() != 3:
            raise ValueError(f"{name} must be [m0][m1][m2]")
        return (ctypes.c_int32 * 3)(*t.shape), ctypes.c_void_p(t.data_ptr())

    def reg_pad(self, img, out=None):
        """Zero padding of an image into the centre of this context's grid."""
        m, p = self._m(img, "img")
        out = self.empty(1) if out is None else out
        _chk(lib().reg_pad(self.handle, m, p, self._t(out, 1, "out")), self.handle, "reg_pad")
        return out

    def reg_crop(self, field, m, out=None):
        """The centred m[0] x m[1] x m[2] block of a field of this context's grid."""
        out = torch.empty(tuple(int(x) for x in m), dtype=self.dtype, device=self.device) if out is None else out
        mm, p = self._m(out, "out")
        _chk(lib().reg_crop(self.handle, mm, self._t(field, 1, "field"), p), self.handle, "reg_crop")
        return out

    def reg_precond(self, r, z=None):
        z = self.empty(3, True) if z is None else z
        _chk(lib().reg_precond(self.handle, self._t(r, 3, "r", True), self._t(z, 3, "z", True)), self.handle,
             "reg_precond")
        return z

    def reg_transport_forward(self, v, rho0, rho1=None):
        rho1 = self.empty(1) if rho1 is None else rho1
        _chk(lib().reg_transport_forward(self.handle, self._t(v, 3, "v", True), self._t(rho0, 1, "rho0"),
                                         self._t(rho1, 1, "rho1")), self.handle, "reg_transport_forward")
        return rho1

    def reg_transport_adjoint(self, v, lam1, lam0=None):
        lam0 = self.empty(1) if lam0 is None else lam0
        _chk(lib().reg_transport_adjoint(self.handle, self._t(v, 3, "v", True), self._t(lam1, 1, "lam1"),
                                         self._t(lam0, 1, "lam0")), self.handle, "reg_transport_adjoint")
        return lam0

    def reg_gradient(self, v, g=None):
        g = self.empty(3, True) if g is None else g
        J, mis, gn = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _chk(lib().reg_gradient(self.handle, self._t(v, 3, "v", True), self._t(g, 3, "g", True), ctypes.byref(J),
                                ctypes.byref(mis), ctypes.byref(gn)), self.handle, "reg_gradient")
        return g, J.value, mis.value, gn.value

    def reg_objective(self, v):
        J, mis = ctypes.c_double(), ctypes.c_double()
        _chk(lib().reg_objective(self.handle, self._t(v, 3, "v", True), ctypes.byref(J), ctypes.byref(mis)),
             self.handle, "reg_objective")
        return J.value, mis.value

    def reg_hessian_matvec(self, vt, Hvt=None):
        Hvt = self.empty(3, True) if Hvt is None else Hvt
        _chk(lib().reg_hessian_matvec(self.handle, self._t(vt, 3, "vt", True), self._t(Hvt, 3, "Hvt", True)),
             self.handle,
             "reg_hessian_matvec")
        return Hvt

    def reg_solve(self, v=None, raise_on_error=True):
        v = torch.zeros((3,) + self.shape, dtype=self.vdtype, device=self.device) if v is None else v
        rep = reg_report()
        st = lib().reg_solve(self.handle, self._t(v, 3, "v", True), ctypes.byref(rep))
        if raise_on_error:
            _chk(st, self.handle, "reg_solve")
        return v, rep.to_dict()

    def reg_deformation(self, v, u=None, want_u=True):
        if want_u and u is None:
            u = self.empty(3)
        mn, mx = ctypes.c_double(), ctypes.c_double()
        _chk(lib().reg_deformation(self.handle, self._t(v, 3, "v", True), self._t(u, 3, "u") if u is not None else None,
                                   ctypes.byref(mn), ctypes.byref(mx)), self.handle, "reg_deformation")
        return u, mn.value, mx.value

    def reg_dot(self, a, b):
        ncomp = a.numel() // self.N
        out = ctypes.c_double()
        _chk(lib().reg_dot(self.handle, ncomp, self._t(a, ncomp, "a", True), self._t(b, ncomp, "b", True),
                           ctypes.byref(out)),
             self.handle, "reg_dot")
        return out.value

    def reg_profile(self, enable=True, every=1):
        """Start (enable) or stop timing launches; every=k times one launch in
        k of each kernel family."""
        _chk(lib().reg_profile(self.handle, int(every) if enable else 0), self.handle, "reg_profile")

    def reg_profile_read(self):
        """{kind: (launches, gpu_ms)} for every kernel family."""
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            n, ms = ctypes.c_int64(), ctypes.c_double()
            _chk(lib().reg_profile_read(self.handle, k, ctypes.byref(n), ctypes.byref(ms)), self.handle,
                 "reg_profile_read")
            out[name] = (n.value, ms.value)
        return out


# ------------------------------------------------------------------ batches
def reg_batch_workspace_size(params_list):
    arr = (reg_params * len(params_list))(*params_list)
    b = ctypes.c_size_t()
    _chk(lib().reg_batch_workspace_size(arr, len(params_list), ctypes.byref(b)), what="reg_batch_workspace_size")
    return b.value


def _bchk(st, b, what):
    if st != REG_OK:
        msg = lib().reg_batch_last_error(b).decode() if b else ""
        raise RegError(st, f"{what}: {msg}")


def _ptrs(ts):
    return (_P * len(ts))(*[ctypes.c_void_p(t.data_ptr()) for t in ts])


class Batch:
    """A reg_batch: independent problems of mixed sizes on one stream (the
    library's own blocking stream unless one is given). contexts[i] is a
    borrowed Context of problem i for the single-problem entry points."""

    def __init__(self, params_list, device="cuda", stream=None):
        self.params = list(params_list)
        self.n = len(self.params)
        self.device = torch.device(device)
        arr = (reg_params * self.n)(*self.params)
        nbytes = reg_batch_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _chk(lib().reg_batch_create(arr, self.n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes, sp,
                                    ctypes.byref(h)), what="reg_batch_create")
        self.handle = h
        self.contexts = []
        for i, p in enumerate(self.params):
            c = ctypes.c_void_p()
            _bchk(lib().reg_batch_ctx(h, i, ctypes.byref(c)), h, "reg_batch_ctx")
            self.contexts.append(Context(p, device, borrowed=c))

    def close(self):
        if self.handle:
            for c in self.contexts:
                c.handle = None
            lib().reg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vel(self, ts, name):
        if len(ts) != self.n:
            raise ValueError(f"{name} needs {self.n} tensors")
        for c, t in zip(self.contexts, ts):
            c._t(t, 3, name, True)
        return _ptrs(ts)

    def _fld(self, ts, name):
        if len(ts) != self.n:
            raise ValueError(f"{name} needs {self.n} tensors")
        for c, t in zip(self.contexts, ts):
            c._t(t, 1, name)
        return _ptrs(ts)

    def reg_set_images(self, i, rho_T, rho_R):
        torch.cuda.synchronize()
        self.contexts[i].reg_set_images(rho_T, rho_R)

    def reg_batch_set_launch(self, blocks=0, chunked=1, use_graph=True):
        _bchk(lib().reg_batch_set_launch(self.handle, int(blocks), int(chunked), int(bool(use_graph))), self.handle,
              "reg_batch_set_launch")

    def reg_batch_set_tile(self, tile1=0, tile2=0):
        """Fixes the tile shape tile1 x tile2 x 64 of the batched canonical launches (0, 0: autotuned)."""
        _bchk(lib().reg_batch_set_tile(self.handle, int(tile1), int(tile2)), self.handle, "reg_batch_set_tile")

    def reg_batch_launch_info(self, mode):
        """(workgroups, chunked, kernel variant, (tile1, tile2), tuned ms) of the last batched launch of a step kind."""
        b, c, v, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        t1, t2 = ctypes.c_int32(), ctypes.c_int32()
        _bchk(lib().reg_batch_launch_info(self.handle, int(mode), ctypes.byref(b), ctypes.byref(c), ctypes.byref(v),
                                          ctypes.byref(t1), ctypes.byref(t2), ctypes.byref(ms)), self.handle,
              "reg_batch_launch_info")
        return b.value, c.value, v.value, (t1.value, t2.value), ms.value

    def reg_batch_stats(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _bchk(lib().reg_batch_stats(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), self.handle,
              "reg_batch_stats")
        return {"batched_launches": a.value, "graph_captures": b.value, "graph_replays": c.value}

    def reg_batch_profile(self, enable=True, every=1):
        _bchk(lib().reg_batch_profile(self.handle, int(every) if enable else 0), self.handle, "reg_batch_profile")

    def reg_batch_profile_read(self):
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            n, ms = ctypes.c_int64(), ctypes.c_double()
            _bchk(lib().reg_batch_profile_read(self.handle, k, ctypes.byref(n), ctypes.byref(ms)), self.handle,
                  "reg_batch_profile_read")
            out[name] = (n.value, ms.value)
        return out

    def reg_batch_transport_forward(self, vs, rho0s, rho1s=None):
        rho1s = [c.empty(1) for c in self.contexts] if rho1s is None else rho1s
        pv, p0, p1 = self._vel(vs, "v"), self._fld(rho0s, "rho0"), self._fld(rho1s, "rho1")
        torch.cuda.synchronize()
        _bchk(lib().reg_batch_transport_forward(self.handle, pv, p0, p1), self.handle, "reg_batch_transport_forward")
        return rho1s

    def reg_batch_gradient(self, vs, gs=None):
        gs = [c.empty(3, True) for c in self.contexts] if gs is None else gs
        pv, pg = self._vel(vs, "v"), self._vel(gs, "g")
        J, mis, gn = (ctypes.c_double * self.n)(), (ctypes.c_double * self.n)(), (ctypes.c_double * self.n)()
        torch.cuda.synchronize()
        _bchk(lib().reg_batch_gradient(self.handle, pv, pg, J, mis, gn), self.handle, "reg_batch_gradient")
        return gs, list(J), list(mis), list(gn)

    def reg_batch_hessian_matvec(self, vts, Hvts=None):
        Hvts = [c.empty(3, True) for c in self.contexts] if Hvts is None else Hvts
        pv, ph = self._vel(vts, "vt"), self._vel(Hvts, "Hvt")
        torch.cuda.synchronize()
        _bchk(lib().reg_batch_hessian_matvec(self.handle, pv, ph), self.handle, "reg_batch_hessian_matvec")
        return Hvts

    def reg_batch_solve(self, vs=None, raise_on_error=True):
        vs = [torch.zeros((3,) + c.shape, dtype=torch.float64, device=self.device) for c in self.contexts] \
            if vs is None else vs
        pv = self._vel(vs, "v")
        reps = (reg_report * self.n)()
        torch.cuda.synchronize()
        st = lib().reg_batch_solve(self.handle, pv, reps)
        if raise_on_error:
            _bchk(st, self.handle, "reg_batch_solve")
        return vs, [r.to_dict() for r in reps]


# ------------------------------------------------------- learned warm start
# (cin, cout, stride) of the network's twelve convolutions, in parameter order
NET_LAYERS = [(2, 16, 1), (16, 16, 1), (16, 32, 2), (32, 32, 1), (32, 64, 2), (64, 64, 1), (64, 64, 1),
              (64, 32, 1), (64, 32, 1), (32, 16, 1), (32, 16, 1), (16, 3, 1)]
NET_LAYER_GRID = [1, 1, 2, 2, 4, 4, 4, 2, 2, 1, 1, 1]  # output grid = n // this


def reg_net_param_count():
    c = ctypes.c_int64()
    _chk(lib().reg_net_param_count(ctypes.byref(c)), what="reg_net_param_count")
    return c.value


def _nchk(st, h, what):
    if st != REG_OK:
        msg = lib().reg_net_last_error(h).decode() if h else ""
        raise RegError(st, f"{what}: {msg}")


class Net:
    """The warm-start network (reg_net) on an n^3 grid."""

    def __init__(self, n=64, device="cuda", stream=None):
        self.n = int(n)
        self.device = torch.device(device)
        self.P = self.n ** 3
        b = ctypes.c_size_t()
        _chk(lib().reg_net_workspace_size(self.n, ctypes.byref(b)), what="reg_net_workspace_size")
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.count = reg_net_param_count()
        h = ctypes.c_void_p()
        _chk(lib().reg_net_create(self.n, ctypes.c_void_p(self.workspace.data_ptr()), b.value, _stream_ptr(stream),
                                  ctypes.byref(h)), what="reg_net_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().reg_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f(self, t, numel, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 CUDA tensor")
        if not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be contiguous with {numel} elements")
        return ctypes.c_void_p(t.data_ptr())

    def reg_net_set_params(self, params):
        _nchk(lib().reg_net_set_params(self.handle, self._f(params, self.count, "params")), self.handle,
              "reg_net_set_params")

    def reg_net_get_params(self):
        out = torch.empty(self.count, dtype=torch.float32, device=self.device)
        _nchk(lib().reg_net_get_params(self.handle, self._f(out, self.count, "params")), self.handle,
              "reg_net_get_params")
        return out

    def reg_net_forward(self, rhoT, rhoR, v=None):
        v = torch.empty((3, self.n, self.n, self.n), dtype=torch.float32, device=self.device) if v is None else v
        _nchk(lib().reg_net_forward(self.handle, self._f(rhoT, self.P, "rho_T"), self._f(rhoR, self.P, "rho_R"),
                                    self._f(v, 3 * self.P, "v")), self.handle, "reg_net_forward")
        return v

    def reg_net_activation(self, layer):
        cin, cout, _ = NET_LAYERS[layer]
        m = self.n // NET_LAYER_GRID[layer]
        out = torch.empty((cout, m, m, m), dtype=torch.float32, device=self.device)
        _nchk(lib().reg_net_activation(self.handle, int(layer), self._f(out, out.numel(), "out")), self.handle,
              "reg_net_activation")
        return out

    def reg_net_loss_grad(self, rhoT, rhoR, target):
        g = torch.empty(self.count, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        _nchk(lib().reg_net_loss_grad(self.handle, self._f(rhoT, self.P, "rho_T"), self._f(rhoR, self.P, "rho_R"),
                                      self._f(target, 3 * self.P, "target"), self._f(g, self.count, "grad"),
                                      ctypes.byref(loss)), self.handle, "reg_net_loss_grad")
        return loss.value, g

    def reg_net_backward(self, dv):
        """dL/dparams for dL/dv = dv after reg_net_forward."""
        g = torch.empty(self.count, dtype=torch.float32, device=self.device)
        _nchk(lib().reg_net_backward(self.handle, self._f(dv, 3 * self.P, "dv"), self._f(g, self.count, "grad")),
              self.handle, "reg_net_backward")
        return g

    def reg_net_step(self, grad, lr=1e-3):
        _nchk(lib().reg_net_step(self.handle, self._f(grad, self.count, "grad"), float(lr)), self.handle,
              "reg_net_step")

    def reg_net_train_step(self, rhoTs, rhoRs, targets, lr=1e-3):
        n = len(rhoTs)
        for t in rhoTs + rhoRs:
            self._f(t, self.P, "image")
        for t in targets:
            self._f(t, 3 * self.P, "target")
        loss = ctypes.c_double()
        _nchk(lib().reg_net_train_step(self.handle, n, _ptrs(rhoTs), _ptrs(rhoRs), _ptrs(targets), float(lr),
                                       ctypes.byref(loss)), self.handle, "reg_net_train_step")
        return loss.value

    def reg_warmstart(self, ctx, v=None):
        """(v, used_fallback, detmin) for a single-precision Context with images set."""
        v = torch.empty((3,) + ctx.shape, dtype=torch.float64, device=self.device) if v is None else v
        fb, dmin = ctypes.c_int32(), ctypes.c_double()
        _chk(lib().reg_warmstart(ctx.handle, self.handle, ctx._t(v, 3, "v", True), ctypes.byref(fb),
                                 ctypes.byref(dmin)), ctx.handle, "reg_warmstart")
        return v, bool(fb.value), dmin.value


def net_params_to_layers(flat):
    """Flat parameter vector (numpy) -> [(W [cout, cin, 3, 3, 3], b [cout])]."""
    out, o = [], 0
    for cin, cout, _ in NET_LAYERS:
        w = flat[o:o + cout * cin * 27].reshape(cout, cin, 3, 3, 3)
        o += cout * cin * 27
        b = flat[o:o + cout]
        o += cout
        out.append((w, b))
    return out


def net_layers_to_params(layers):
    import numpy as np

    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])
