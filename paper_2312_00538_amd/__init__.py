"""Python binding of the MI355X ANOVA-NFFT / interior-point SVM library.

Argument marshalling only: every step of the computation runs in the HIP
library `libanova_nfft.so` (C ABI declared in include/anova_nfft.h). torch is
used for device memory and streams. Importing works without a GPU; creating a
plan needs the built library and a visible gfx950 device, and fails loudly
otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libanova_nfft.so")

OK, INVALID_ARG, OUT_OF_MEMORY, HIP_ERROR, NOT_CONVERGED, NUMERICAL = range(6)
PREC_FP64, PREC_MIXED = 0, 1
PRECOND_NONE, PRECOND_PCHOL, PRECOND_NYSTROM, PRECOND_DIAG, PRECOND_RPCHOL, PRECOND_RFF = 0, 1, 2, 3, 4, 5
KRYLOV_MINRES, KRYLOV_GMRES = 0, 1

EXPORTED = [
    "anova_opts_default", "anova_plan_create", "anova_matvec", "anova_plan_destroy",
    "anova_plan_info", "anova_ipm_opts_default", "svm_ipm_solve", "anova_pivoted_cholesky",
    "anova_nystrom", "anova_last_error", "anova_profile_begin", "anova_profile_end",
    "anova_server_opts_default", "anova_server_create", "anova_server_submit", "anova_server_wait",
    "anova_server_counters", "anova_server_destroy", "anova_request_footprint", "anova_grid_solve",
    "anova_tune_opts_default", "anova_autotune", "anova_rp_cholesky", "anova_decision_function",
    "anova_rff_factor", "anova_mi_windows", "anova_matvec_noalloc", "anova_kaiser_bessel",
    "anova_axis_coefficients", "anova_lowrank_apply",
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
                ("err_tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("graphs", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("factor_fp32", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("max_active", ctypes.c_int32), ("hbm_budget", ctypes.c_int64),
                ("share_launches", ctypes.c_int32), ("reserved", ctypes.c_int32), ("gather_us", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("labels", ctypes.c_void_p), ("windows", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("N", ctypes.c_int64), ("d", ctypes.c_int32), ("P", ctypes.c_int32),
                ("C", ctypes.c_double), ("nfft", ctypes.c_void_p), ("ipm", ctypes.c_void_p)]


class IpmStats(ctypes.Structure):
    _fields_ = [("ip_iters", ctypes.c_int32), ("kry_iters_total", ctypes.c_int32),
                ("kry_iters_max", ctypes.c_int32), ("rank_used", ctypes.c_int32), ("status", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("mu", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("dual_obj", ctypes.c_double), ("primal_obj", ctypes.c_double),
                ("xi_alpha_rel", ctypes.c_double), ("xi_lambda_rel", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class GridProblem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("labels", ctypes.c_void_p), ("n_c", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("C", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("lambda_", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("rhs", ctypes.c_int32), ("target_rel_err", ctypes.c_double),
                ("precisions", ctypes.c_int32), ("reps", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class TuneCandidate(ctypes.Structure):
    _fields_ = [("n_bw", ctypes.c_int32), ("cutoff_m", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seg_points", ctypes.c_int32), ("rel_err", ctypes.c_double), ("ms", ctypes.c_double)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32), ("footprint", ctypes.c_int64),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("stats", IpmStats)]


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
        "anova_matvec_noalloc": ([P, P, i32, i64, P, i64, P], ctypes.c_int),
        "anova_kaiser_bessel": ([ctypes.POINTER(Opts), P, i32, P, P], ctypes.c_int),
        "anova_axis_coefficients": ([dbl, dbl, dbl, ctypes.POINTER(Opts), P, P, P, ctypes.POINTER(i32)], ctypes.c_int),
        "anova_plan_destroy": ([P], ctypes.c_int),
        "anova_plan_info": ([P, ctypes.POINTER(PlanInfo)], ctypes.c_int),
        "anova_ipm_opts_default": ([ctypes.POINTER(IpmOpts)], ctypes.c_int),
        "svm_ipm_solve": ([P, P, dbl, ctypes.POINTER(IpmOpts), P, ctypes.POINTER(dbl),
                           ctypes.POINTER(IpmStats), P], ctypes.c_int),
        "anova_pivoted_cholesky": ([P, i32, dbl, P, i64, P, ctypes.POINTER(i32), P], ctypes.c_int),
        "anova_nystrom": ([P, P, i32, i64, P, i64, P], ctypes.c_int),
        "anova_lowrank_apply": ([i64, i32, P, i64, P, P, P, i32, P, P], ctypes.c_int),
        "anova_last_error": ([], ctypes.c_char_p),
        "anova_profile_begin": ([P], ctypes.c_int),
        "anova_profile_end": ([P, P, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "anova_server_opts_default": ([ctypes.POINTER(ServerOpts)], ctypes.c_int),
        "anova_server_create": ([ctypes.POINTER(ServerOpts), i32, ctypes.POINTER(P)], ctypes.c_int),
        "anova_server_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(i64)], ctypes.c_int),
        "anova_server_wait": ([P, i64, P, ctypes.POINTER(ServerResult)], ctypes.c_int),
        "anova_server_counters": ([P, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "anova_server_destroy": ([P], ctypes.c_int),
        "anova_request_footprint": ([i64, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(IpmOpts),
                                     ctypes.POINTER(i64)], ctypes.c_int),
        "anova_grid_solve": ([ctypes.POINTER(GridProblem), i32, ctypes.POINTER(IpmOpts), i32, dbl,
                              ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "anova_tune_opts_default": ([ctypes.POINTER(TuneOpts)], ctypes.c_int),
        "anova_rp_cholesky": ([P, i32, dbl, P, P, i64, P, ctypes.POINTER(i32), P], ctypes.c_int),
        "anova_rff_factor": ([P, i32, P, P, P, i64, P], ctypes.c_int),
        "anova_decision_function": ([P, i64, i64, P, i64, i64, i32, P, i32, P, P, ctypes.POINTER(Opts), P, P,
                                     dbl, P, P], ctypes.c_int),
        "anova_autotune": ([P, i64, i32, i64, P, i32, P, P, ctypes.POINTER(TuneOpts), P, ctypes.POINTER(Opts),
                            ctypes.POINTER(TuneCandidate), i32, ctypes.POINTER(i32)], ctypes.c_int),
        "anova_mi_windows": ([P, i64, i32, i64, P, i32, i32, P, P, P], ctypes.c_int),
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


@contextlib.contextmanager
def _on_stream(stream, *inputs):
    """Runs the binding's own copies and allocations on the stream that the
    library call gets, and yields that stream's handle. With an explicit
    `stream` other than torch's current one, `stream` first waits for the
    current stream (which produced the inputs), and the inputs are recorded on
    it so that the caching allocator keeps their memory until the library's
    asynchronous reads on `stream` are done."""
    import torch
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        yield ctypes.c_void_p(cur.cuda_stream)
        return
    stream.wait_stream(cur)
    for t in inputs:
        if t is not None:
            t.record_stream(stream)
    with torch.cuda.stream(stream):
        yield ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    return t


def _set_fields(o, kw):
    fields = {f[0] for f in type(o)._fields_}
    for k, v in kw.items():
        if k not in fields:
            raise TypeError(f"unknown {type(o).__name__} field {k!r}")
        setattr(o, k, v)


def default_opts(**kw) -> Opts:
    lib = load_library()
    o = Opts()
    _check(lib.anova_opts_default(ctypes.byref(o)))
    _set_fields(o, kw)
    return o


def default_ipm_opts(**kw) -> IpmOpts:
    lib = load_library()
    o = IpmOpts()
    _check(lib.anova_ipm_opts_default(ctypes.byref(o)))
    _set_fields(o, kw)
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
        return self._matvec(_lib.anova_matvec, x, out, stream)

    def matvec_noalloc(self, x, out=None, stream=None):
        """y = K x through anova_matvec_noalloc (one-vector passes, scratch in
        the library's static per-device array; no device allocation in the
        library call)."""
        return self._matvec(_lib.anova_matvec_noalloc, x, out, stream)

    def _matvec(self, fn, x, out, stream):
        import torch
        x = _dev_f64(x, "x")
        vec = x.dim() == 1
        with _on_stream(stream, x, out) as s:
            xm = x.reshape(self.N, 1) if vec else x
            R = int(xm.shape[1])
            xc = xm.t().contiguous()               # R x N, column r contiguous
            if out is None:
                yc = torch.empty((R, self.N), dtype=torch.float64, device=x.device)
            else:
                yc = out.reshape(self.N, R).t() if not vec else out.reshape(1, self.N)
                if not yc.is_contiguous():
                    raise ValueError("out must be column-contiguous")
            _check(fn(self._h, ctypes.c_void_p(xc.data_ptr()), R, self.N, ctypes.c_void_p(yc.data_ptr()), self.N, s))
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
        labels = _dev_f64(labels, "labels")
        if opts is None:
            opts = default_ipm_opts(**kw)
        with _on_stream(stream, labels) as s:
            labels = labels.contiguous()
            alpha = torch.empty(self.N, dtype=torch.float64, device=labels.device)
            lam = ctypes.c_double(0.0)
            st = IpmStats()
            rc = _lib.svm_ipm_solve(self._h, ctypes.c_void_p(labels.data_ptr()), float(C), ctypes.byref(opts),
                                    ctypes.c_void_p(alpha.data_ptr()), ctypes.byref(lam), ctypes.byref(st), s)
        _check(rc, allow=(OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return alpha, lam.value, st.as_dict()

    def pivoted_cholesky(self, rank: int, err_tol: float = 0.0, stream=None):
        import torch
        piv = np.zeros(rank, dtype=np.int64)
        used = ctypes.c_int32(0)
        with _on_stream(stream) as s:
            L = torch.empty((rank, self.N), dtype=torch.float64, device=self.device)
            _check(_lib.anova_pivoted_cholesky(self._h, rank, float(err_tol), ctypes.c_void_p(L.data_ptr()),
                                               self.N, piv.ctypes.data_as(ctypes.c_void_p), ctypes.byref(used), s))
        r = used.value
        return L[:r].t(), piv[:r]

    def rp_cholesky(self, uniforms, err_tol: float = 0.0, stream=None):
        """Randomly pivoted Cholesky with the given draws (one per step, in [0, 1))."""
        import torch
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).reshape(-1))
        rank = int(u.shape[0])
        piv = np.zeros(rank, dtype=np.int64)
        used = ctypes.c_int32(0)
        with _on_stream(stream) as s:
            L = torch.empty((rank, self.N), dtype=torch.float64, device=self.device)
            _check(_lib.anova_rp_cholesky(self._h, rank, float(err_tol), u.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.c_void_p(L.data_ptr()), self.N, piv.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(used), s))
        r = used.value
        return L[:r].t(), piv[:r]

    def rff_factor(self, w, b, stream=None):
        """Random Fourier features Z (N x k) for draws w (k x 3) and b (k)."""
        import torch
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1, 3))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
        k = int(b.shape[0])
        with _on_stream(stream) as s:
            Z = torch.empty((k, self.N), dtype=torch.float64, device=self.device)
            _check(_lib.anova_rff_factor(self._h, k, w.ctypes.data_as(ctypes.c_void_p),
                                         b.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(Z.data_ptr()), self.N, s))
        return Z.t()

    def nystrom(self, G, stream=None):
        import torch
        G = _dev_f64(G, "G")
        k = int(G.shape[1])
        with _on_stream(stream, G) as s:
            Gc = G.t().contiguous()
            Z = torch.empty((k, self.N), dtype=torch.float64, device=G.device)
            _check(_lib.anova_nystrom(self._h, ctypes.c_void_p(Gc.data_ptr()), k, self.N,
                                      ctypes.c_void_p(Z.data_ptr()), self.N, s))
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


def kaiser_bessel(u, opts: Opts | None = None):
    """(phi(u) / phi(0), phi_hat(k) for k = 0..n/2) of the plans' Kaiser-Bessel
    window (anova_kaiser_bessel); host only."""
    lib = load_library()
    o = opts if opts is not None else default_opts()
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
    phi = np.zeros(u.shape[0])
    ph = np.zeros(o.oversample * o.n_bw // 2 + 1)
    _check(lib.anova_kaiser_bessel(ctypes.byref(o), u.ctypes.data_as(ctypes.c_void_p), int(u.shape[0]),
                                   phi.ctypes.data_as(ctypes.c_void_p), ph.ctypes.data_as(ctypes.c_void_p)))
    return phi, ph


def axis_coefficients(lo: float, hi: float, sigma: float, opts: Opts | None = None):
    """Per-axis coefficients a plan builds (anova_axis_coefficients); host only.
    Returns dict(bk (k = -n_bw/2 .. n_bw/2 - 1), circ, center, scale, sigma_a,
    kerr, reg_p)."""
    lib = load_library()
    o = opts if opts is not None else default_opts()
    bk = np.zeros(o.n_bw)
    circ = np.zeros(o.oversample * o.n_bw)
    ax = np.zeros(4)
    rp = ctypes.c_int32(0)
    _check(lib.anova_axis_coefficients(float(lo), float(hi), float(sigma), ctypes.byref(o),
                                       bk.ctypes.data_as(ctypes.c_void_p), circ.ctypes.data_as(ctypes.c_void_p),
                                       ax.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rp)))
    return dict(bk=bk, circ=circ, center=ax[0], scale=ax[1], sigma_a=ax[2], kerr=ax[3], reg_p=rp.value)


def lowrank_apply(Zt, theta, r, y=None, fp32_products: bool = False, stream=None):
    """(Theta + Y Z Z^T Y)^{-1} r through the solver's preconditioner kernels
    (anova_lowrank_apply). Zt: (k, N) device FP64, row j = column j of Z;
    theta, r, y: (N,) device FP64 (y None = identity)."""
    import torch
    lib = load_library()
    Zt = _dev_f64(Zt, "Zt")
    theta, r = _dev_f64(theta, "theta"), _dev_f64(r, "r")
    k, N = int(Zt.shape[0]), int(Zt.shape[1])
    with _on_stream(stream, r) as s:
        Zc, th, rc = Zt.contiguous(), theta.contiguous(), r.contiguous()
        yc = _dev_f64(y, "y").contiguous() if y is not None else None
        out = torch.empty(N, dtype=torch.float64, device=r.device)
        _check(lib.anova_lowrank_apply(N, k, ctypes.c_void_p(Zc.data_ptr()), N, ctypes.c_void_p(th.data_ptr()),
                                       ctypes.c_void_p(yc.data_ptr()) if yc is not None else None,
                                       ctypes.c_void_p(rc.data_ptr()), 1 if fp32_products else 0,
                                       ctypes.c_void_p(out.data_ptr()), s))
    return out


def request_footprint(N: int, d: int, P: int, nfft: Opts | None = None, ipm: IpmOpts | None = None) -> int:
    """Device bytes the server charges for a request of this shape."""
    lib = load_library()
    b = ctypes.c_int64(0)
    _check(lib.anova_request_footprint(int(N), int(d), int(P), ctypes.byref(nfft) if nfft else None,
                                       ctypes.byref(ipm) if ipm else None, ctypes.byref(b)))
    return b.value


def decision_function(X, Xnew, windows, sigma, labels, alpha, lam: float, eta=None, opts: Opts | None = None,
                      stream=None, **opt_kw):
    """f(Xnew) = sum_j alpha_j y_j k(x, x_j) - lam (anova_decision_function);
    X, Xnew row-major device tensors, labels and alpha device vectors."""
    import torch
    lib = load_library()
    X = _dev_f64(X, "X")
    Xn = _dev_f64(Xnew, "Xnew")
    if X.dim() != 2 or Xn.dim() != 2 or X.stride(1) != 1 or Xn.stride(1) != 1 or X.shape[1] != Xn.shape[1]:
        raise ValueError("X and Xnew must be 2-D row-major tensors with the same number of columns")
    labels = _dev_f64(labels, "labels")
    alpha = _dev_f64(alpha, "alpha")
    win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 3))
    Pw = int(win.shape[0])
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (Pw,)))
    et = None if eta is None else np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float64), (Pw,)))
    if opts is None:
        opts = default_opts(**opt_kw)
    M = int(Xn.shape[0])
    with _on_stream(stream, X, Xn, labels, alpha) as s:
        labels = labels.contiguous()
        alpha = alpha.contiguous()
        f = torch.empty(M, dtype=torch.float64, device=Xn.device)
        _check(lib.anova_decision_function(ctypes.c_void_p(X.data_ptr()), int(X.shape[0]), X.stride(0),
                                           ctypes.c_void_p(Xn.data_ptr()), M, Xn.stride(0), int(X.shape[1]),
                                           win.ctypes.data_as(ctypes.c_void_p), Pw,
                                           sig.ctypes.data_as(ctypes.c_void_p),
                                           et.ctypes.data_as(ctypes.c_void_p) if et is not None else None,
                                           ctypes.byref(opts), ctypes.c_void_p(labels.data_ptr()),
                                           ctypes.c_void_p(alpha.data_ptr()), float(lam),
                                           ctypes.c_void_p(f.data_ptr()), s))
    return f


def mi_windows(X, labels, bins: int = 32, P: int | None = None, stream=None):
    """Windows of features by mutual-information ranking (anova_mi_windows).
    X: device N x d row-major tensor; labels: device N tensor (class by sign).
    Returns (windows P x 3 int32, -1 padded; mutual-information estimate per
    feature). P defaults to ceil(d / 3)."""
    lib = load_library()
    X = _dev_f64(X, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D row-major tensor")
    y = _dev_f64(labels, "labels")
    N, d = int(X.shape[0]), int(X.shape[1])
    if y.shape != (N,):
        raise ValueError("labels must have shape (N,)")
    P = (d + 2) // 3 if P is None else int(P)
    win = np.full((max(P, 1), 3), -1, dtype=np.int32)
    mi = np.zeros(d, dtype=np.float64)
    with _on_stream(stream, X, y) as s:
        y = y.contiguous()
        _check(lib.anova_mi_windows(ctypes.c_void_p(X.data_ptr()), N, d, X.stride(0), ctypes.c_void_p(y.data_ptr()),
                                    int(bins), P, win.ctypes.data_as(ctypes.c_void_p),
                                    mi.ctypes.data_as(ctypes.c_void_p), s))
    return win[:P], mi


def autotune(X, windows, sigma, eta=None, target_rel_err: float = 1e-4, rhs: int = 1,
             precisions=("fp64", "mixed"), reps: int = 3, seed: int = 0, stream=None):
    """Choose the fast-summation options for this data set (anova_autotune).
    Returns (Opts, candidates, chosen index); candidates are dicts with n_bw,
    cutoff_m, precision, seg_points, rel_err (< 0: size not usable) and ms
    (< 0: not timed). Raises AnovaError(NOT_CONVERGED) when nothing reaches
    the target."""
    lib = load_library()
    X = _dev_f64(X, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D row-major tensor")
    N, d = int(X.shape[0]), int(X.shape[1])
    win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 3))
    Pw = int(win.shape[0])
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (Pw,)))
    et = None if eta is None else np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float64), (Pw,)))
    t = TuneOpts()
    _check(lib.anova_tune_opts_default(ctypes.byref(t)))
    t.rhs, t.target_rel_err, t.reps, t.seed = int(rhs), float(target_rel_err), int(reps), int(seed)
    t.precisions = (1 if "fp64" in precisions else 0) | (2 if "mixed" in precisions else 0)
    best = Opts()
    cands = (TuneCandidate * 64)()
    n = ctypes.c_int32(0)
    rc = lib.anova_autotune(ctypes.c_void_p(X.data_ptr()), N, d, X.stride(0), win.ctypes.data_as(ctypes.c_void_p),
                            Pw, sig.ctypes.data_as(ctypes.c_void_p),
                            et.ctypes.data_as(ctypes.c_void_p) if et is not None else None, ctypes.byref(t),
                            _stream(stream), ctypes.byref(best), cands, 64, ctypes.byref(n))
    out = [{f[0]: getattr(cands[i], f[0]) for f in TuneCandidate._fields_} for i in range(min(n.value, 64))]
    _check(rc)
    chosen = next(i for i, c in enumerate(out) if c["n_bw"] == best.n_bw and c["cutoff_m"] == best.cutoff_m
                  and c["precision"] == best.precision and c["seg_points"] == best.seg_points)
    return best, out, chosen


def grid_solve(problems, opts: IpmOpts | None = None, max_active: int = 64, gather_us: float = 200.0,
               **kw):
    """Hyperparameter grid of IPM solves (anova_grid_solve).

    problems: list of (plan, labels, Cs) with labels a device tensor of the
    plan's N and Cs a sequence of C values; each plan in one problem only.
    Returns (results, launches, matvecs) with results[i] = (alpha (N x nC
    device tensor, column j for Cs[j]), lambdas (nC,), stats (list of dicts,
    'status' per solve)). Runs on the current device; waits for torch's
    current stream before it starts."""
    import torch
    lib = load_library()
    if opts is None:
        opts = default_ipm_opts(**kw)
    arr = (GridProblem * len(problems))()
    keep = []
    for i, (plan, labels, Cs) in enumerate(problems):
        labels = _dev_f64(labels, "labels").contiguous()
        c = np.ascontiguousarray(np.asarray(Cs, dtype=np.float64).reshape(-1))
        nc = int(c.shape[0])
        alpha = torch.empty((nc, plan.N), dtype=torch.float64, device=labels.device)
        lam = np.zeros(nc, dtype=np.float64)
        st = (IpmStats * max(nc, 1))()
        keep.append((labels, c, alpha, lam, st))
        arr[i] = GridProblem(plan.handle.value, labels.data_ptr(), nc, 0, c.ctypes.data, alpha.data_ptr(),
                             lam.ctypes.data, ctypes.addressof(st))
    torch.cuda.current_stream().synchronize()
    la, mv = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib.anova_grid_solve(arr, len(problems), ctypes.byref(opts), int(max_active), float(gather_us),
                                ctypes.byref(la), ctypes.byref(mv)))
    out = []
    for (labels, c, alpha, lam, st) in keep:
        out.append((alpha.t(), lam.copy(), [st[j].as_dict() for j in range(len(c))]))
    return out, la.value, mv.value


class Server:
    """Continuous-batching request server for IPM solves on one GPU (host
    inputs are copied at submit; results come back on the host)."""

    def __init__(self, max_active: int = 8, hbm_budget: int = 0, share_launches: bool = True,
                 gather_us: float = 200.0, device: int = 0):
        lib = load_library()
        o = ServerOpts()
        _check(lib.anova_server_opts_default(ctypes.byref(o)))
        o.max_active, o.hbm_budget = int(max_active), int(hbm_budget)
        o.share_launches, o.gather_us = int(bool(share_launches)), float(gather_us)
        h = ctypes.c_void_p()
        _check(lib.anova_server_create(ctypes.byref(o), int(device), ctypes.byref(h)))
        self._h = h
        self._n = {}

    def submit(self, X, labels, windows, sigma, C: float, nfft: Opts | None = None, ipm: IpmOpts | None = None,
               **ipm_kw) -> int:
        X = np.ascontiguousarray(X, dtype=np.float64)
        y = np.ascontiguousarray(labels, dtype=np.float64)
        win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 3))
        P = int(win.shape[0])
        sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (P,)))
        if ipm is None and ipm_kw:
            ipm = default_ipm_opts(**ipm_kw)
        q = Request(X.ctypes.data, y.ctypes.data, win.ctypes.data, sig.ctypes.data, X.shape[0], X.shape[1], P,
                    float(C), ctypes.cast(ctypes.pointer(nfft), ctypes.c_void_p) if nfft else None,
                    ctypes.cast(ctypes.pointer(ipm), ctypes.c_void_p) if ipm else None)
        t = ctypes.c_int64(0)
        _check(_lib.anova_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._n[t.value] = X.shape[0]
        return t.value

    def wait(self, ticket: int, allow_not_converged: bool = True):
        """Blocks until the solve is done; returns (alpha, result dict)."""
        alpha = np.empty(self._n.pop(ticket), dtype=np.float64)
        r = ServerResult()
        rc = _lib.anova_server_wait(self._h, int(ticket), alpha.ctypes.data_as(ctypes.c_void_p), ctypes.byref(r))
        _check(rc, allow=(OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        res = {"status": r.status, "footprint": r.footprint, "queue_ms": r.queue_ms, "run_ms": r.run_ms,
               "latency_ms": r.latency_ms, "lambda": r.lambda_, "stats": r.stats.as_dict()}
        return alpha, res

    def counters(self) -> tuple[int, int]:
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib.anova_server_counters(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.anova_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
