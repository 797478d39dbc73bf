"""Thin ctypes binding of liblincoll (C ABI in include/lincoll.h).

Argument marshalling only: every step of the operator runs in the HIP
library.  Device arrays are torch tensors (contiguous, on the plan's GPU);
the binding passes their data pointers and torch's current HIP stream.
If the library is missing the import of this module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblincoll.so")

OK, EINVAL, ENOMEM, EHIP, ENOTREADY, ENOTIMPL, EDIVERGED, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
DTYPES = {"f64": 0, "f32": 1, "bf16x3": 2}
PATHS = {"auto": 0, "staged": 1, "fused": 2}
TABLES = {"g": 0, "W": 1, "Phi": 2, "Omega": 3, "phi": 4}
INFO = {"n": 0, "J": 1, "R": 2, "dtype": 3, "path": 4, "maxw_batch": 5, "device_bytes": 6,
        "hip_error": 7, "eps": 8, "graph": 9, "fused_per_cu": 10, "tuned_ms": 11, "L": 12, "project": 13,
        "quad_fix": 14, "zblock": 15, "plane_tile": 16, "tune_cached": 17, "fused_ppt": 18,
        "fused_keep": 19, "last_path": 20, "fused_split": 21}
PRECONDS = {"none": 0, "sweep": 1, "learned": 2}
INNERS = {"gmres": 0, "source": 1}
MLP_IN, MLP_HIDDEN, MLP_OUT = 26, 128, 5
MLP_WEIGHTS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_OUT + MLP_OUT
OPTIONS = {"graph": 0, "fused_per_cu": 1, "path": 2, "sphere_polar": 3, "sphere_azimuth": 4, "project": 5,
           "quad_fix": 6, "zblock": 7, "plane_tile": 8, "tune_cache": 9, "fused_ppt": 10,
           "fused_keep": 11, "check_finite": 12, "fused_split": 13}
SYMBOLS = ["lincoll_params_default", "lincoll_plan", "lincoll_plan_ex", "lincoll_set_stream",
           "lincoll_set_maxwellians", "lincoll_apply", "lincoll_project", "quadcoll_apply",
           "lincoll_get_info", "lincoll_destroy", "lincoll_strerror", "lincoll_plan_tables",
           "lincoll_set_option", "lincoll_autotune", "lincoll_rk4", "lincoll_steady_default",
           "lincoll_steady_residual", "lincoll_steady_newton_apply", "lincoll_steady_solve",
           "lincoll_steady_precondition",
           "lincoll_mlp_create", "lincoll_mlp_destroy", "lincoll_mlp_set_stream", "lincoll_mlp_weights",
           "lincoll_mlp_forward", "lincoll_mlp_loss_grad", "lincoll_mlp_train", "lincoll_learned_features",
           "lincoll_learned_correction", "lincoll_debug_fail_alloc", "lincoll_apply_noalloc"]


class LincollError(RuntimeError):
    def __init__(self, status, what, hip_error=None):
        extra = f", hipError {hip_error}" if hip_error else ""
        super().__init__(f"{what}: {_lib.lincoll_strerror(status).decode()} ({status}{extra})")
        self.status = status
        self.hip_error = hip_error


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_double), ("omega", ctypes.c_double),
                ("C", ctypes.c_double), ("R", ctypes.c_double), ("J", ctypes.c_int),
                ("eps", ctypes.c_double), ("quad_rule", ctypes.c_int), ("project", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("dtype", ctypes.c_int), ("path", ctypes.c_int)]


class SteadyParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("x_l", ctypes.c_double), ("x_r", ctypes.c_double),
                ("kn", ctypes.c_double), ("mass", ctypes.c_double), ("theta_l", ctypes.c_double),
                ("theta_r", ctypes.c_double), ("u_l", ctypes.c_double * 3), ("u_r", ctypes.c_double * 3),
                ("tol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("inner_atol", ctypes.c_double),
                ("max_newton", ctypes.c_int), ("max_inner", ctypes.c_int), ("restart", ctypes.c_int),
                ("init", ctypes.c_int), ("precond", ctypes.c_int), ("inner", ctypes.c_int),
                ("backtrack", ctypes.c_int), ("mlp", ctypes.c_void_p),
                ("rec_X", ctypes.c_void_p), ("rec_T", ctypes.c_void_p), ("rec_cap", ctypes.c_int)]


class SteadyReport(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("inner_iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("residual", ctypes.c_double), ("mass", ctypes.c_double),
                ("res_history", ctypes.c_double * 65), ("inner_history", ctypes.c_int * 64),
                ("ms_total", ctypes.c_double), ("ms_residual", ctypes.c_double), ("ms_inner", ctypes.c_double),
                ("rec_rows", ctypes.c_int), ("backtracks", ctypes.c_int)]

    def as_dict(self):
        k = min(self.newton_iters, 64)
        return {"newton_iters": self.newton_iters, "inner_iters": self.inner_iters,
                "converged": bool(self.converged), "residual": self.residual, "mass": self.mass,
                "res_history": list(self.res_history[:k + 1]), "inner_history": list(self.inner_history[:k]),
                "ms_total": self.ms_total, "ms_residual": self.ms_residual, "ms_inner": self.ms_inner,
                "rec_rows": self.rec_rows, "backtracks": self.backtracks}


def steady_params(nx, **kw):
    """SteadyParams with the library defaults for nx cells, then kw
    (u_l / u_r as 3-sequences, precond as a name, mlp as an MLP, rec_X /
    rec_T as float32 CUDA tensors [rows, 26] / [rows, 5], which the caller
    keeps alive)."""
    sp = SteadyParams()
    _lib.lincoll_steady_default(ctypes.byref(sp), int(nx))
    if "rec_X" in kw:
        X, T = kw.pop("rec_X"), kw.pop("rec_T")
        if X.shape[0] != T.shape[0] or X.shape[1:] != (MLP_IN,) or T.shape[1:] != (MLP_OUT,):
            raise ValueError("rec_X [rows, 26] and rec_T [rows, 5] expected")
        sp.rec_X, sp.rec_T, sp.rec_cap = X.data_ptr(), T.data_ptr(), X.shape[0]
    for k, v in kw.items():
        if k == "mlp":
            v = v._h.value if v is not None else None
        if k in ("u_l", "u_r"):
            v = (ctypes.c_double * 3)(*[float(a) for a in v])
        if k == "precond" and isinstance(v, str):
            v = PRECONDS[v]
        if k == "inner" and isinstance(v, str):
            v = INNERS[v]
        setattr(sp, k, v)
    return sp


def _load():
    # torch bundles its own HIP runtime with the same soname as the system
    # one the library links; whichever is loaded first serves the process.
    # Load torch's first so that the library and torch share one runtime
    # (loading the library first left hipGetDevice without a device).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblincoll.so not built at {LIB_PATH}; run python -m paper_2503_09580_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "lincoll_params_default": (None, [P(Params), i, d, d, i]),
        "lincoll_plan": (i, [i, d, d, i, P(vp)]),
        "lincoll_plan_ex": (i, [P(Params), P(vp)]),
        "lincoll_set_stream": (i, [vp, vp]),
        "lincoll_set_maxwellians": (i, [vp, vp, i]),
        "lincoll_apply": (i, [vp, vp, vp, i]),
        "lincoll_apply_noalloc": (i, [vp, vp, vp, i]),
        "lincoll_project": (i, [vp, vp, vp, i]),
        "quadcoll_apply": (i, [vp, vp, vp, i]),
        "lincoll_get_info": (i, [vp, i, P(d)]),
        "lincoll_destroy": (None, [vp]),
        "lincoll_strerror": (ctypes.c_char_p, [i]),
        "lincoll_debug_fail_alloc": (None, [i]),
        "lincoll_plan_tables": (ctypes.c_longlong, [P(Params), i, P(d), ctypes.c_longlong]),
        "lincoll_set_option": (i, [vp, i, i]),
        "lincoll_autotune": (i, [vp, vp, vp, i, i]),
        "lincoll_rk4": (i, [vp, vp, i, d, i]),
        "lincoll_steady_default": (None, [P(SteadyParams), i]),
        "lincoll_steady_residual": (i, [vp, P(SteadyParams), vp, vp, P(d)]),
        "lincoll_steady_newton_apply": (i, [vp, P(SteadyParams), vp, vp, vp]),
        "lincoll_steady_solve": (i, [vp, P(SteadyParams), vp, P(SteadyReport)]),
        "lincoll_steady_precondition": (i, [vp, P(SteadyParams), vp, vp, vp]),
        "lincoll_mlp_create": (i, [ctypes.c_ulonglong, P(vp)]),
        "lincoll_mlp_destroy": (None, [vp]),
        "lincoll_mlp_set_stream": (i, [vp, vp]),
        "lincoll_mlp_weights": (i, [vp, P(ctypes.c_float), ctypes.c_longlong, i]),
        "lincoll_mlp_forward": (i, [vp, vp, vp, i]),
        "lincoll_mlp_loss_grad": (i, [vp, vp, vp, i, vp, P(d)]),
        "lincoll_mlp_train": (i, [vp, vp, vp, i, i, d, P(d)]),
        "lincoll_learned_features": (i, [vp, P(SteadyParams), vp, vp, vp, P(d)]),
        "lincoll_learned_correction": (i, [vp, P(SteadyParams), vp, vp, d, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def make_params(n, L, omega, dtype="f64", **kw):
    p = Params()
    _lib.lincoll_params_default(ctypes.byref(p), int(n), float(L), float(omega), DTYPES[dtype])
    for k, v in kw.items():
        if k == "path":
            v = PATHS[v] if isinstance(v, str) else v
        setattr(p, k, v)
    return p


def plan_tables(n, L, omega, table, **kw):
    """Host-only plan table (no GPU): g, W, Phi, Omega or phi."""
    p = make_params(n, L, omega, "f64", **kw)
    cnt = _lib.lincoll_plan_tables(ctypes.byref(p), TABLES[table], None, 0)
    if cnt < 0:
        raise LincollError(int(cnt), "lincoll_plan_tables")
    out = np.empty(cnt, dtype=np.float64)
    st = _lib.lincoll_plan_tables(ctypes.byref(p), TABLES[table], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cnt)
    if st < 0:
        raise LincollError(int(st), "lincoll_plan_tables")
    return out


def _check(st, what):
    if st != OK:
        hip = None
        if st == EHIP:
            v = ctypes.c_double()
            if _lib.lincoll_get_info(None, INFO["hip_error"], ctypes.byref(v)) == OK:
                hip = int(v.value)
        raise LincollError(st, what, hip)


class Plan:
    """A lincoll plan on the current GPU.

    Plan(n, L, omega, dtype="f64"|"f32"|"bf16x3", **params) with optional
    C, R, J, eps, quad_rule, project, max_batch, path ("auto"|"staged"|"fused").
    """

    def __init__(self, n, L, omega, dtype="f64", **kw):
        import torch
        self._torch = torch
        self.n, self.L, self.omega, self.dtype = n, L, omega, dtype
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        self._p = make_params(n, L, omega, dtype, **kw)
        self._h = ctypes.c_void_p()
        _check(_lib.lincoll_plan_ex(ctypes.byref(self._p), ctypes.byref(self._h)), "lincoll_plan_ex")
        self._stream = None

    def close(self):
        if self._h:
            _lib.lincoll_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = self._torch.cuda.current_stream().cuda_stream
        if s != self._stream:
            _check(_lib.lincoll_set_stream(self._h, ctypes.c_void_p(s)), "lincoll_set_stream")
            self._stream = s

    def _dev(self, t, dtype, shape_tail=None, name="array"):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
        if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [batch, {shape_tail}]")
        return ctypes.c_void_p(t.data_ptr())

    def set_maxwellians(self, params):
        """params: float64 CUDA tensor [batch, 5] = (rho, u1, u2, u3, theta)."""
        self._sync_stream()
        self._params_ref = params
        _check(_lib.lincoll_set_maxwellians(self._h, self._dev(params, self._torch.float64, (5,), "params"),
                                            params.shape[0]), "lincoll_set_maxwellians")

    def apply(self, h, out=None):
        n = self.n
        if out is None:
            out = self._torch.empty_like(h)
        self._sync_stream()
        _check(_lib.lincoll_apply(self._h, self._dev(h, self.tdtype, (n, n, n), "h"),
                                  self._dev(out, self.tdtype, (n, n, n), "out"), h.shape[0]), "lincoll_apply")
        return out

    def apply_noalloc(self, h, out):
        """lincoll_apply_noalloc: out must be preallocated (nothing is
        allocated, by the library or here)."""
        n = self.n
        self._sync_stream()
        _check(_lib.lincoll_apply_noalloc(self._h, self._dev(h, self.tdtype, (n, n, n), "h"),
                                          self._dev(out, self.tdtype, (n, n, n), "out"), h.shape[0]),
               "lincoll_apply_noalloc")
        return out

    def project(self, x, y=None):
        n = self.n
        if y is None:
            y = self._torch.empty_like(x)
        self._sync_stream()
        _check(_lib.lincoll_project(self._h, self._dev(x, self.tdtype, (n, n, n), "x"),
                                    self._dev(y, self.tdtype, (n, n, n), "y"), x.shape[0]), "lincoll_project")
        return y

    def set_option(self, key, value):
        """lincoll_set_option: key is a name in OPTIONS (the LINCOLL_OPT_* of
        include/lincoll.h, e.g. "graph" 0|1, "fused_per_cu", "fused_keep",
        "fused_split" 0 = by batch | 1 = never | S parts); "path" takes
        "auto" | "staged" | "fused"."""
        v = PATHS[value] if key == "path" else int(value)
        _check(_lib.lincoll_set_option(self._h, OPTIONS[key], v), "lincoll_set_option")

    def autotune(self, h, out=None, reps=3):
        """Times every supported launch configuration on (h, out) and keeps the
        fastest (or takes the process-wide cached choice for the same device,
        n, dtype and batch bucket); returns its milliseconds per apply.  out
        receives L[h] when timing ran."""
        n = self.n
        if out is None:
            out = self._torch.empty_like(h)
        self._sync_stream()
        _check(_lib.lincoll_autotune(self._h, self._dev(h, self.tdtype, (n, n, n), "h"),
                                     self._dev(out, self.tdtype, (n, n, n), "out"), h.shape[0], int(reps)),
               "lincoll_autotune")
        return self.info("tuned_ms")

    def quadcoll(self, f, out=None):
        """Q(f, f) by eq. (14) for a float64 CUDA tensor [batch, n, n, n]."""
        n = self.n
        torch = self._torch
        if out is None:
            out = torch.empty_like(f)
        self._sync_stream()
        _check(_lib.quadcoll_apply(self._h, self._dev(f, torch.float64, (n, n, n), "f"),
                                   self._dev(out, torch.float64, (n, n, n), "out"), f.shape[0]), "quadcoll_apply")
        return out

    def rk4(self, f, dt, steps):
        """Advances f (contiguous [batch, n, n, n] tensor of the plan's dtype)
        in place by `steps` RK4 steps of df/dt = L[f]."""
        n = self.n
        self._sync_stream()
        _check(_lib.lincoll_rk4(self._h, self._dev(f, self.tdtype, (n, n, n), "f"), f.shape[0], float(dt),
                                int(steps)), "lincoll_rk4")
        return f

    def _field(self, t, name):
        n = self.n
        if t.dim() != 4 or tuple(t.shape[1:]) != (n, n, n):
            raise ValueError(f"{name} must be [nx, {n}, {n}, {n}]")
        return self._dev(t, self._torch.float64, None, name)

    def steady_residual(self, sp, f, r=None):
        """(r, norm): residual of the steady problem sp (SteadyParams) at f
        (float64 CUDA tensor [nx, n, n, n])."""
        if r is None:
            r = self._torch.empty_like(f)
        v = ctypes.c_double()
        self._sync_stream()
        _check(_lib.lincoll_steady_residual(self._h, ctypes.byref(sp), self._field(f, "f"), self._field(r, "r"),
                                            ctypes.byref(v)), "lincoll_steady_residual")
        return r, v.value

    def steady_newton_apply(self, sp, f, g, out=None):
        """out = T[g] - P L P g / Kn about the local Maxwellians of f."""
        if out is None:
            out = self._torch.empty_like(g)
        self._sync_stream()
        _check(_lib.lincoll_steady_newton_apply(self._h, ctypes.byref(sp), self._field(f, "f"), self._field(g, "g"),
                                                self._field(out, "out")), "lincoll_steady_newton_apply")
        return out

    def steady_precondition(self, sp, f, y, z=None):
        """z = the inner solver's preconditioner applied to y about the local Maxwellians of f."""
        if z is None:
            z = self._torch.empty_like(y)
        self._sync_stream()
        _check(_lib.lincoll_steady_precondition(self._h, ctypes.byref(sp), self._field(f, "f"), self._field(y, "y"),
                                                self._field(z, "z")), "lincoll_steady_precondition")
        return z

    def steady_solve(self, sp, f):
        """Modified Newton solve in place on f; returns the report as a dict."""
        rep = SteadyReport()
        self._sync_stream()
        _check(_lib.lincoll_steady_solve(self._h, ctypes.byref(sp), self._field(f, "f"), ctypes.byref(rep)),
               "lincoll_steady_solve")
        return rep.as_dict()

    def learned_features(self, sp, f, z):
        """(X float32 [nx, 26], s): features of z about the local Maxwellians of f."""
        torch = self._torch
        X = torch.empty((f.shape[0], MLP_IN), dtype=torch.float32, device=f.device)
        v = ctypes.c_double()
        self._sync_stream()
        _check(_lib.lincoll_learned_features(self._h, ctypes.byref(sp), self._field(f, "f"), self._field(z, "z"),
                                             ctypes.c_void_p(X.data_ptr()), ctypes.byref(v)), "lincoll_learned_features")
        return X, v.value

    def learned_correction(self, sp, f, Y, s):
        """sum_a s Y_a M_c psi_a about the local Maxwellians of f."""
        out = self._torch.empty_like(f)
        if Y.dtype != self._torch.float32 or not Y.is_contiguous() or tuple(Y.shape) != (f.shape[0], MLP_OUT):
            raise ValueError("Y must be a contiguous float32 [nx, 5] tensor")
        self._sync_stream()
        _check(_lib.lincoll_learned_correction(self._h, ctypes.byref(sp), self._field(f, "f"),
                                               ctypes.c_void_p(Y.data_ptr()), float(s), self._field(out, "out")),
               "lincoll_learned_correction")
        return out

    def info(self, key):
        """lincoll_get_info: key is a name in INFO (the LINCOLL_INFO_* of
        include/lincoll.h, e.g. "path", "last_path", "fused_split")."""
        v = ctypes.c_double()
        _check(_lib.lincoll_get_info(self._h, INFO[key], ctypes.byref(v)), "lincoll_get_info")
        return v.value


class MLP:
    """The learned correction's network (26 -> 128 tanh -> 5, FP32) on the
    current GPU; arrays are float32 CUDA tensors."""

    def __init__(self, seed=0):
        import torch
        self._torch = torch
        self._h = ctypes.c_void_p()
        _check(_lib.lincoll_mlp_create(int(seed), ctypes.byref(self._h)), "lincoll_mlp_create")

    def close(self):
        if self._h:
            _lib.lincoll_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync(self):
        _check(_lib.lincoll_mlp_set_stream(self._h, ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)),
               "lincoll_mlp_set_stream")

    @staticmethod
    def _f32(t, cols, name):
        if not t.is_cuda or not t.is_contiguous() or t.dtype.itemsize != 4 or t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor [rows, {cols}]")
        return ctypes.c_void_p(t.data_ptr())

    def get_weights(self):
        w = np.empty(MLP_WEIGHTS, dtype=np.float32)
        self._sync()
        _check(_lib.lincoll_mlp_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), MLP_WEIGHTS, 0),
               "lincoll_mlp_weights")
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != MLP_WEIGHTS:
            raise ValueError(f"{MLP_WEIGHTS} weights expected")
        self._sync()
        _check(_lib.lincoll_mlp_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), MLP_WEIGHTS, 1),
               "lincoll_mlp_weights")

    def forward(self, X):
        Y = self._torch.empty((X.shape[0], MLP_OUT), dtype=self._torch.float32, device=X.device)
        self._sync()
        _check(_lib.lincoll_mlp_forward(self._h, self._f32(X, MLP_IN, "X"), self._f32(Y, MLP_OUT, "Y"), X.shape[0]),
               "lincoll_mlp_forward")
        return Y

    def loss_grad(self, X, T):
        g = self._torch.empty(MLP_WEIGHTS, dtype=self._torch.float32, device=X.device)
        v = ctypes.c_double()
        self._sync()
        _check(_lib.lincoll_mlp_loss_grad(self._h, self._f32(X, MLP_IN, "X"), self._f32(T, MLP_OUT, "T"), X.shape[0],
                                          ctypes.c_void_p(g.data_ptr()), ctypes.byref(v)), "lincoll_mlp_loss_grad")
        return v.value, g

    def train(self, X, T, steps, lr=1e-3):
        v = ctypes.c_double()
        self._sync()
        _check(_lib.lincoll_mlp_train(self._h, self._f32(X, MLP_IN, "X"), self._f32(T, MLP_OUT, "T"), X.shape[0],
                                      int(steps), float(lr), ctypes.byref(v)), "lincoll_mlp_train")
        return v.value
