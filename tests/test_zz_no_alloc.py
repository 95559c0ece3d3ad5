"""anova_matvec_noalloc (the allocation-free matvec) against anova_matvec,
called through the C ABI: two calls in a row, the second on a smaller plan,
each equal to the allocating entry point's result (bit for bit for one
right-hand side, where both run the same one-vector kernels; to rounding for
several, which anova_matvec batches) and within the matvec bar of the FP64
direct-sum oracle; plans whose scratch exceeds the static array are rejected
with INVALID_ARG."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
import paper_2312_00538_amd as lib
from gpu_util import device, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _call(fn, plan, x, R):
    import torch
    y = torch.full((R, plan.N), float("nan"), dtype=torch.float64, device=x.device)
    xc = x.t().contiguous() if R > 1 else x.reshape(1, plan.N).contiguous()
    s = torch.cuda.current_stream()
    rc = fn(plan.handle, ctypes.c_void_p(xc.data_ptr()), R, plan.N, ctypes.c_void_p(y.data_ptr()), plan.N,
            ctypes.c_void_p(s.cuda_stream))
    assert rc == lib.OK, lib.load_library().anova_last_error()
    torch.cuda.synchronize()
    return y.cpu().numpy().T


@pytest.mark.parametrize("precision", [lib.PREC_FP64, lib.PREC_MIXED])
def test_noalloc_matvec_equals_matvec_on_two_calls(precision):
    dev = device()
    L = lib.load_library()
    cases = [(3000, 9, 2, 11), (1100, 6, 1, 12)]  # (N, d, R, seed): the second call is smaller
    for N, d, R, seed in cases:
        p = workloads.small_plain(seed=seed, N=N, d=d, R=R)
        plan = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma, precision=precision)
        x = to_dev(p.v, dev)
        y_ref = _call(L.anova_matvec, plan, x, R)
        y_na = _call(L.anova_matvec_noalloc, plan, x, R)
        print(f"noalloc N={N} d={d} R={R} precision={precision}", flush=True)
        if R == 1:
            # the same kernels in the same order on the same plan
            assert np.array_equal(y_na, y_ref)
        else:
            # anova_matvec takes R >= 2 through the 16-wide batched kernels
            # (other summation orders; FP32 contractions for mixed plans)
            bar = 1e-11 if precision == lib.PREC_FP64 else 1e-5
            assert max(rel_l2(y_na[:, r], y_ref[:, r]) for r in range(R)) <= bar
        for r in range(R):
            ref = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v[:, r])
            assert rel_l2(y_na[:, r], ref) <= 1e-4
        plan.close()


def test_noalloc_rejects_plans_beyond_the_scratch_maximum():
    dev = device()
    L = lib.load_library()
    N, d = 1_200_000, 12  # 4 windows: the permuted input and gathered values alone need 76.8 MB
    rng = np.random.default_rng(3)
    X = rng.uniform(-0.25, 0.25, size=(N, d))
    win = [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]]
    plan = lib.Plan(to_dev(X, dev), win, 1.0)
    import torch
    x = torch.ones(N, dtype=torch.float64, device=dev)
    y = torch.zeros(N, dtype=torch.float64, device=dev)
    rc = L.anova_matvec_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), 1, N, ctypes.c_void_p(y.data_ptr()), N,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == lib.INVALID_ARG
    assert b"allocation-free maximum" in L.anova_last_error()
    plan.close()
