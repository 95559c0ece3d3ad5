"""The C-ABI library loads on the CPU and exports every entry point that
include/anova_nfft.h declares; option defaults match Table 1; argument checks
that run before any device work return INVALID_ARG (no GPU needed)."""
import ctypes
import json
import os
import re

import pytest

import paper_2312_00538_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "anova_nfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lib.LIB_PATH):
        from paper_2312_00538_amd import build
        build.build(verbose=False)
    return lib.load_library()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 10
    assert sorted(names) == sorted(lib.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_defaults_follow_table1(L):
    t = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_parameters.json")))
    o = lib.default_ipm_opts()
    assert o.sigma_bar == t["barrier_reduction"]
    assert o.gamma0 == t["step_to_boundary"]
    assert o.mu0 == t["mu0"]
    assert o.max_kry == t["max_krylov_iterations"]
    assert o.tol_kry == t["krylov_tolerance"]
    assert o.err_tol == t["cholesky_err_tol"]
    assert o.tol_inf == t["ipm_tolerance"]
    n = lib.default_opts()
    assert (n.n_bw, n.oversample, n.cutoff_m, n.eps_b) == (32, 2, 4, 0.25)


def test_invalid_arguments_are_rejected_before_device_work(L):
    h = ctypes.c_void_p()
    o = lib.default_opts()
    import numpy as np
    win = np.array([[0, 1, 2]], dtype=np.int32)
    sig = np.array([1.0])
    fake = ctypes.c_void_p(0x1000)
    args = lambda N, d, ldx, w, P, s: (fake, N, d, ldx, w.ctypes.data_as(ctypes.c_void_p), P,
                                       s.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(o), None,
                                       ctypes.byref(h))
    assert L.anova_plan_create(*args(0, 3, 3, win, 1, sig)) == lib.INVALID_ARG
    assert L.anova_plan_create(*args(10, 3, 2, win, 1, sig)) == lib.INVALID_ARG
    bad = np.array([[0, 0, 1]], dtype=np.int32)
    assert L.anova_plan_create(*args(10, 3, 3, bad, 1, sig)) == lib.INVALID_ARG
    assert b"repeated" in L.anova_last_error()
    bad = np.array([[0, 5, -1]], dtype=np.int32)
    assert L.anova_plan_create(*args(10, 3, 3, bad, 1, sig)) == lib.INVALID_ARG
    empty = np.array([[-1, -1, -1]], dtype=np.int32)
    assert L.anova_plan_create(*args(10, 3, 3, empty, 1, sig)) == lib.INVALID_ARG
    assert L.anova_plan_create(*args(10, 3, 3, win, 1, np.array([0.0]))) == lib.INVALID_ARG
    o.cutoff_m = 9
    assert L.anova_plan_create(*args(10, 3, 3, win, 1, sig)) == lib.INVALID_ARG
    o.cutoff_m = 4
    o.version = 99
    assert L.anova_plan_create(*args(10, 3, 3, win, 1, sig)) == lib.INVALID_ARG
    assert L.anova_matvec(None, fake, 1, 10, fake, 10, None) == lib.INVALID_ARG
    assert L.anova_plan_destroy(None) == lib.OK


def test_server_options_and_footprint(L):
    # defaults of the request server, and the footprint it charges: grows with
    # the problem and with the Nystrom build's extra N x k buffers
    o = lib.ServerOpts()
    assert L.anova_server_opts_default(ctypes.byref(o)) == lib.OK
    assert (o.max_active, o.hbm_budget, o.share_launches, o.gather_us) == (8, 0, 1, 200.0)
    f = lib.request_footprint
    assert f(10_000, 9, 3) < f(100_000, 9, 3) < f(100_000, 30, 10)
    assert f(100_000, 9, 3) > 100_000 * 9 * 8          # at least the data itself
    ny = lib.default_ipm_opts(precond=lib.PRECOND_NYSTROM)
    assert f(100_000, 9, 3, ipm=ny) > f(100_000, 9, 3)
    b = ctypes.c_int64(0)
    assert L.anova_request_footprint(0, 9, 3, None, None, ctypes.byref(b)) == lib.INVALID_ARG
    assert L.anova_server_destroy(None) == lib.OK
    t = ctypes.c_int64(0)
    assert L.anova_server_submit(None, None, ctypes.byref(t)) == lib.INVALID_ARG


def test_grid_solve_rejects_bad_arguments(L):
    # checked before any device work: no problems, a NULL plan
    assert L.anova_grid_solve(None, 1, None, 8, 200.0, None, None) == lib.INVALID_ARG
    probs = (lib.GridProblem * 1)()
    assert L.anova_grid_solve(probs, 0, None, 8, 200.0, None, None) == lib.INVALID_ARG
    assert L.anova_grid_solve(probs, 1, None, 8, 200.0, None, None) == lib.INVALID_ARG
    assert b"NULL plan" in L.anova_last_error()
    o = lib.default_ipm_opts()
    o.version = 99
    assert L.anova_grid_solve(probs, 1, ctypes.byref(o), 8, 200.0, None, None) == lib.INVALID_ARG


def test_autotune_options_and_argument_checks(L):
    t = lib.TuneOpts()
    assert L.anova_tune_opts_default(ctypes.byref(t)) == lib.OK
    assert (t.rhs, t.target_rel_err, t.precisions, t.reps) == (1, 1e-4, 3, 3)
    best = lib.Opts()
    fake = ctypes.c_void_p(0x1000)
    import numpy as np
    win = np.array([[0, 1, 2]], dtype=np.int32)
    sig = np.array([1.0])
    args = (fake, 10, 3, 3, win.ctypes.data_as(ctypes.c_void_p), 1, sig.ctypes.data_as(ctypes.c_void_p), None)
    assert L.anova_autotune(*args, None, None, None, None, 0, None) == lib.INVALID_ARG   # NULL best
    t.version = 99
    assert L.anova_autotune(*args, ctypes.byref(t), None, ctypes.byref(best), None, 0, None) == lib.INVALID_ARG
    t.version = lib.TuneOpts().version or 1
    t.rhs = 0
    assert L.anova_autotune(*args, ctypes.byref(t), None, ctypes.byref(best), None, 0, None) == lib.INVALID_ARG


def test_mi_windows_argument_checks(L):
    # sizes are checked before any device access: fake device pointers suffice
    import numpy as np
    fake = ctypes.c_void_p(0x1000)
    win = np.zeros((4, 3), dtype=np.int32)
    w = win.ctypes.data_as(ctypes.c_void_p)
    ok = dict(N=100, d=9, ldx=9, bins=32, P=3)
    for bad in (dict(N=0), dict(d=0), dict(ldx=8), dict(bins=1), dict(bins=1025), dict(P=0), dict(P=4)):
        a = {**ok, **bad}
        rc = L.anova_mi_windows(fake, a["N"], a["d"], a["ldx"], fake, a["bins"], a["P"], w, None, None)
        assert rc == lib.INVALID_ARG, bad
        assert L.anova_last_error()
    assert L.anova_mi_windows(None, 100, 9, 9, fake, 32, 3, w, None, None) == lib.INVALID_ARG
    assert L.anova_mi_windows(fake, 100, 9, 9, fake, 32, 3, None, None, None) == lib.INVALID_ARG
