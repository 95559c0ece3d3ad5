"""Python binding of the MI355X ANOVA-NFFT / interior-point SVM library.

Argument marshalling only: every step of the computation runs in the HIP
library `libanova_nfft.so` (C ABI declared in include/anova_nfft.h). torch is
used for device memory and streams. Importing works without a GPU; creating a
plan needs the built library and a visible gfx950 device, and fails loudly
otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libanova_nfft.so")

OK, INVALID_ARG, OUT_OF_MEMORY, HIP_ERROR, NOT_CONVERGED, NUMERICAL = range(6)
PREC_FP64, PREC_MIXED = 0, 1
PRECOND_NONE, PRECOND_PCHOL, PRECOND_NYSTROM = 0, 1, 2

EXPORTED = [
    "anova_opts_default", "anova_plan_create", "anova_matvec", "anova_plan_destroy",
    "anova_plan_info", "anova_ipm_opts_default", "svm_ipm_solve", "anova_pivoted_cholesky",
    "anova_nystrom", "anova_last_error", "anova_profile_begin", "anova_profile_end",
]
STAGES = ["permute", "spread", "fold", "convolve", "gather", "window_sum"]


class AnovaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("n_bw", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("cutoff_m", ctypes.c_int32), ("eps_b", ctypes.c_double), ("reg_p", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seg_points", ctypes.c_int32), ("batch_min_rhs", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_windows", ctypes.c_int32), ("n_segments", ctypes.c_int32),
                ("cutoff_m", ctypes.c_int32), ("precision", ctypes.c_int32), ("eps_b", ctypes.c_double),
                ("max_kernel_err", ctypes.c_double), ("grid_cells", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64)]


class IpmOpts(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("max_ip", ctypes.c_int32), ("max_kry", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("tol", ctypes.c_double), ("tol_inf", ctypes.c_double),
                ("tol_kry", ctypes.c_double), ("sigma_bar", ctypes.c_double), ("gamma0", ctypes.c_double),
                ("mu0", ctypes.c_double), ("rank", ctypes.c_int32), ("mu_rule", ctypes.c_int32),
                ("err_tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class IpmStats(ctypes.Structure):
    _fields_ = [("ip_iters", ctypes.c_int32), ("kry_iters_total", ctypes.c_int32),
                ("kry_iters_max", ctypes.c_int32), ("rank_used", ctypes.c_int32), ("status", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("mu", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("dual_obj", ctypes.c_double), ("primal_obj", ctypes.c_double),
                ("xi_alpha_rel", ctypes.c_double), ("xi_lambda_rel", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2312_00538_amd.build` "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "anova_opts_default": ([ctypes.POINTER(Opts)], ctypes.c_int),
        "anova_plan_create": ([P, i64, i32, i64, P, i32, P, P, ctypes.POINTER(Opts), P, ctypes.POINTER(P)],
                              ctypes.c_int),
        "anova_matvec": ([P, P, i32, i64, P, i64, P], ctypes.c_int),
        "anova_plan_destroy": ([P], ctypes.c_int),
        "anova_plan_info": ([P, ctypes.POINTER(PlanInfo)], ctypes.c_int),
        "anova_ipm_opts_default": ([ctypes.POINTER(IpmOpts)], ctypes.c_int),
        "svm_ipm_solve": ([P, P, dbl, ctypes.POINTER(IpmOpts), P, ctypes.POINTER(dbl),
                           ctypes.POINTER(IpmStats), P], ctypes.c_int),
        "anova_pivoted_cholesky": ([P, i32, dbl, P, i64, P, ctypes.POINTER(i32), P], ctypes.c_int),
        "anova_nystrom": ([P, P, i32, i64, P, i64, P], ctypes.c_int),
        "anova_last_error": ([], ctypes.c_char_p),
        "anova_profile_begin": ([P], ctypes.c_int),
        "anova_profile_end": ([P, P, i32, ctypes.POINTER(i32)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        msg = _lib.anova_last_error().decode() if _lib is not None else ""
        raise AnovaError(rc, msg)
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    return t


def default_opts(**kw) -> Opts:
    lib = load_library()
    o = Opts()
    _check(lib.anova_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_ipm_opts(**kw) -> IpmOpts:
    lib = load_library()
    o = IpmOpts()
    _check(lib.anova_ipm_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Plan:
    """Fast-summation plan of K = sum_l eta_l K_l for one data matrix."""

    def __init__(self, X, windows, sigma, eta=None, opts: Opts | None = None, stream=None, **opt_kw):
        import torch
        lib = load_library()
        X = _dev_f64(X, "X")
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be a 2-D row-major tensor")
        self.N, self.d = int(X.shape[0]), int(X.shape[1])
        win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 3))
        self.P = int(win.shape[0])
        sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (self.P,)))
        et = None if eta is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(eta, dtype=np.float64), (self.P,)))
        if opts is None:
            opts = default_opts(**opt_kw)
        self.opts = opts
        h = ctypes.c_void_p()
        rc = lib.anova_plan_create(ctypes.c_void_p(X.data_ptr()), self.N, self.d, X.stride(0),
                                   win.ctypes.data_as(ctypes.c_void_p), self.P,
                                   sig.ctypes.data_as(ctypes.c_void_p),
                                   et.ctypes.data_as(ctypes.c_void_p) if et is not None else None,
                                   ctypes.byref(opts), _stream(stream), ctypes.byref(h))
        _check(rc)
        self._h = h
        self.device = X.device

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = PlanInfo()
        _check(_lib.anova_plan_info(self._h, ctypes.byref(inf)))
        return {f[0]: getattr(inf, f[0]) for f in PlanInfo._fields_}

    def matvec(self, x, out=None, stream=None):
        """y = K x for x of shape (N,) or (N, R) (R columns, column-major: x.T contiguous)."""
        import torch
        x = _dev_f64(x, "x")
        vec = x.dim() == 1
        xm = x.reshape(self.N, 1) if vec else x
        R = int(xm.shape[1])
        xc = xm.t().contiguous()               # R x N, column r contiguous
        if out is None:
            yc = torch.empty((R, self.N), dtype=torch.float64, device=x.device)
        else:
            yc = out.reshape(self.N, R).t() if not vec else out.reshape(1, self.N)
            if not yc.is_contiguous():
                raise ValueError("out must be column-contiguous")
        _check(_lib.anova_matvec(self._h, ctypes.c_void_p(xc.data_ptr()), R, self.N,
                                 ctypes.c_void_p(yc.data_ptr()), self.N, _stream(stream)))
        y = yc.t()
        return y.reshape(self.N) if vec else y

    def profile_begin(self):
        _check(_lib.anova_profile_begin(self._h))

    def profile_end(self) -> tuple[dict, int]:
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int32(0)
        _check(_lib.anova_profile_end(self._h, ms, len(STAGES), ctypes.byref(n)))
        return {s: ms[i] for i, s in enumerate(STAGES)}, n.value

    def matvec_raw(self, x_ptr: int, R: int, ldx: int, y_ptr: int, ldy: int, stream=None):
        _check(_lib.anova_matvec(self._h, ctypes.c_void_p(x_ptr), R, ldx, ctypes.c_void_p(y_ptr), ldy,
                                 _stream(stream)))

    def solve(self, labels, C: float, opts: IpmOpts | None = None, stream=None, allow_not_converged=False,
              **kw):
        """Interior point SVM training; returns (alpha, lambda, stats dict)."""
        import torch
        labels = _dev_f64(labels, "labels").contiguous()
        if opts is None:
            opts = default_ipm_opts(**kw)
        alpha = torch.empty(self.N, dtype=torch.float64, device=labels.device)
        lam = ctypes.c_double(0.0)
        st = IpmStats()
        rc = _lib.svm_ipm_solve(self._h, ctypes.c_void_p(labels.data_ptr()), float(C), ctypes.byref(opts),
                                ctypes.c_void_p(alpha.data_ptr()), ctypes.byref(lam), ctypes.byref(st),
                                _stream(stream))
        _check(rc, allow=(OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return alpha, lam.value, st.as_dict()

    def pivoted_cholesky(self, rank: int, err_tol: float = 0.0, stream=None):
        import torch
        L = torch.empty((rank, self.N), dtype=torch.float64, device=self.device)
        piv = np.zeros(rank, dtype=np.int64)
        used = ctypes.c_int32(0)
        _check(_lib.anova_pivoted_cholesky(self._h, rank, float(err_tol), ctypes.c_void_p(L.data_ptr()),
                                           self.N, piv.ctypes.data_as(ctypes.c_void_p), ctypes.byref(used),
                                           _stream(stream)))
        r = used.value
        return L[:r].t(), piv[:r]

    def nystrom(self, G, stream=None):
        import torch
        G = _dev_f64(G, "G")
        k = int(G.shape[1])
        Gc = G.t().contiguous()
        Z = torch.empty((k, self.N), dtype=torch.float64, device=G.device)
        _check(_lib.anova_nystrom(self._h, ctypes.c_void_p(Gc.data_ptr()), k, self.N,
                                  ctypes.c_void_p(Z.data_ptr()), self.N, _stream(stream)))
        return Z.t()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.anova_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
