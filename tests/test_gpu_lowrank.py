"""The IPM's preconditioner apply on its own (Section 5): anova_lowrank_apply
computes (Theta + Y Z Z^T Y)^{-1} r with the kernels every IPM iteration runs
(capacitance matrix on the FP64 matrix cores, its Cholesky factor, the two
N x k passes and the triangular solves between them). Each case is compared
with the oracle's Woodbury form, which the CPU tests pin against a dense
inverse.

Inputs are shaped like an IPM iteration's: Z with column norms falling
geometrically from about sqrt(N) to 1e-3 (a pivoted-Cholesky factor of a
smooth kernel), Theta log-uniform over 1e-4..1e4 (barrier weights of free rows
and of rows at a bound), y random signs. Both sides evaluate the same formula
in FP64 with different summation orders. The capacitance matrix's condition
number reaches 1e7 here, but the output is dominated by Theta^{-1} r: the
oracle's FP64 result and the same formula in 80-bit arithmetic differ by about
1e-15 in relative l2 norm for these inputs (N up to 20000, k = 200), so the bar
is 1e-11. A wrong entry of the Cholesky factor, a dropped partial sum or a
transposed operand moves the result by far more."""
import numpy as np
import pytest

import oracle
from gpu_util import device, rel_l2, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def dev():
    return device()


def _case(seed, N, k, theta_range=(1e-4, 1e4)):
    rng = np.random.default_rng(seed)
    scale = np.sqrt(N) * np.geomspace(1.0, 1e-3 / np.sqrt(N), k) if k > 1 else np.array([np.sqrt(N)])
    Zt = rng.standard_normal((N, k)) * (scale / np.sqrt(N))[None, :]     # N x k, column norms ~ scale
    theta = np.exp(rng.uniform(np.log(theta_range[0]), np.log(theta_range[1]), N))
    y = np.where(rng.random(N) < 0.5, -1.0, 1.0)
    r = rng.standard_normal(N)
    return Zt, theta, y, r


# k: one column, one 16-row block, a ragged block count, the workloads' rank,
# the largest rank held in registers and one past it; N: several SYRK row chunks
# with a ragged tail at the largest size
@pytest.mark.parametrize("N,k", [(3000, 1), (3000, 16), (3000, 37), (5000, 200), (5000, 256), (4000, 300),
                                 (70001, 200)])
@pytest.mark.parametrize("fp32", [False, True])
def test_lowrank_apply_matches_the_woodbury_oracle(dev, N, k, fp32):
    import paper_2312_00538_amd as lib
    Zt, theta, y, r = _case(N + k, N, k)
    Zr = Zt.astype(np.float32).astype(np.float64) if fp32 else Zt
    ref = oracle.woodbury_apply(theta, y, Zr, r)
    out = lib.lowrank_apply(to_dev(np.ascontiguousarray(Zt.T), dev), to_dev(theta, dev), to_dev(r, dev),
                            y=to_dev(y, dev), fp32_products=fp32).cpu().numpy()
    err = rel_l2(out, ref)
    print(f"N={N} k={k} fp32={fp32}: rel l2 {err:.2e}")
    assert err <= TOL


def test_lowrank_apply_identity_signs_and_repeat(dev):
    # y = NULL means Y = I; two calls in a row give the same bits
    import paper_2312_00538_amd as lib
    Zt, theta, _, r = _case(5, 2000, 50)
    ref = oracle.woodbury_apply(theta, np.ones(2000), Zt, r)
    args = (to_dev(np.ascontiguousarray(Zt.T), dev), to_dev(theta, dev), to_dev(r, dev))
    a = lib.lowrank_apply(*args).cpu().numpy()
    b = lib.lowrank_apply(*args).cpu().numpy()
    assert rel_l2(a, ref) <= TOL
    assert np.array_equal(a, b)


def test_lowrank_apply_rejects_bad_sizes(dev):
    import paper_2312_00538_amd as lib
    import torch
    Zt = torch.zeros((1025, 100), dtype=torch.float64, device=dev)
    v = torch.ones(100, dtype=torch.float64, device=dev)
    with pytest.raises(lib.AnovaError) as e:
        lib.lowrank_apply(Zt, v, v)
    assert e.value.status == lib.INVALID_ARG
