"""GPU parity of the FP64 batched matvec (16 right-hand sides per pass, FP64
matrix-core spreading and gathering on v_mfma_f64_16x16x4f64, FP64 grids and
window sums) against the FP64 direct-sum oracle of Section 3's kernel sum, and
against the FP64 one-vector kernels of the same plan (the same approximation
through independent code, so the two agree to FP64 rounding)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, rel_l2, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4          # the matvec bar
TOL_FP64 = 1e-6     # FP64 plans at m = 4, bandwidth 32: approximation error ~1e-7
TOL_ROUND = 1e-11   # batched FP64 against one-vector FP64: summation order only
FP64 = 0


@pytest.fixture(scope="module")
def dev():
    return device()


def _plan(p, dev, sigma=None, **kw):
    import paper_2312_00538_amd as lib
    return lib.Plan(to_dev(p.X, dev), p.windows, p.sigma if sigma is None else sigma, precision=FP64, **kw)


def test_two_passes_with_ragged_tail(dev):
    # R = 20: one full pass of 16 and a pass of 4
    p = workloads.small_plain(seed=3, N=2000, d=9, R=20)
    pl = _plan(p, dev)
    y = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    ref = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v)
    errs = [rel_l2(y[:, r], ref[:, r]) for r in range(20)]
    print("rel_l2 per rhs", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL_FP64
    y1 = _plan(p, dev, batch_min_rhs=-1).matvec(to_dev(p.v, dev)).cpu().numpy()
    d = max(rel_l2(y[:, r], y1[:, r]) for r in range(20))
    print(f"FP64 batched vs one-vector kernels: {d:.2e}")
    assert d <= TOL_ROUND


@pytest.mark.parametrize("n_bw,sigma", [(24, 0.7), (24, 1.3), (40, 0.9), (16, 2.0), (48, 0.5)])
def test_bandwidths_and_grid_boxes_of_any_size(dev, n_bw, sigma):
    p = workloads.gaussian_mixture(seed=9, N=1200, d=9, sigma=sigma, R=16)
    pl = _plan(p, dev, n_bw=n_bw)
    y = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    y1 = _plan(p, dev, n_bw=n_bw, batch_min_rhs=-1).matvec(to_dev(p.v, dev)).cpu().numpy()
    d = max(rel_l2(y[:, r], y1[:, r]) for r in range(16))
    print(f"n_bw={n_bw} sigma={sigma} grid_cells={pl.info()['grid_cells']} FP64 batched vs one-vector {d:.2e}")
    assert d <= TOL_ROUND


@pytest.mark.parametrize("N,d,sigma,seed,R", [(37, 5, 0.5, 1, 3), (513, 7, 0.25, 2, 16), (1000, 4, 4.0, 3, 2),
                                              (3001, 3, 1.0, 4, 17), (257, 1, 0.3, 5, 5), (800, 2, 0.7, 6, 9)])
def test_ragged_shapes_and_window_kinds(dev, N, d, sigma, seed, R):
    p = workloads.gaussian_mixture(seed=seed, N=N, d=d, sigma=sigma, R=R)
    pl = _plan(p, dev)
    y = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    ref = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v)
    errs = [rel_l2(y[:, r], ref[:, r]) for r in range(R)]
    y1 = _plan(p, dev, batch_min_rhs=-1).matvec(to_dev(p.v, dev)).cpu().numpy()
    d = max(rel_l2(y[:, r], y1[:, r]) for r in range(R))
    print(f"N={N} d={d} sigma={sigma} R={R} windows={p.windows.tolist()} max rel_l2={max(errs):.3e}, "
          f"vs one-vector {d:.2e}")
    assert max(errs) <= TOL
    assert d <= TOL_ROUND


def test_weights_per_window_sigma_and_leading_dims(dev):
    import paper_2312_00538_amd as lib
    import torch
    p = workloads.gaussian_mixture(seed=7, N=1500, d=8, R=6)
    sig = np.array([0.3, 0.9, 2.0])
    eta = np.array([0.5, 1.5, -0.25])
    pl = lib.Plan(to_dev(p.X, dev), p.windows, sig, eta=eta, precision=FP64)
    ref = oracle.anova_matvec(p.X, p.windows, sig, p.v, eta=eta)
    N, R, ldx, ldy = 1500, 6, 1531, 1600
    xb = torch.zeros(R * ldx, dtype=torch.float64, device=dev)
    yb = torch.full((R * ldy,), 7.0, dtype=torch.float64, device=dev)
    for r in range(R):
        xb[r * ldx:r * ldx + N] = to_dev(p.v[:, r], dev)
    pl.matvec_raw(xb.data_ptr(), R, ldx, yb.data_ptr(), ldy)
    torch.cuda.synchronize()
    yh = yb.cpu().numpy()
    for r in range(R):
        assert rel_l2(yh[r * ldy:r * ldy + N], ref[:, r]) <= TOL
        assert np.all(yh[r * ldy + N:(r + 1) * ldy] == 7.0)


def test_rhs_independent_of_batch_companions(dev):
    # each right-hand side goes through its own rows of every contraction (and
    # its own half of the right-hand sides), so a column's result is
    # bit-identical whether it runs alone or among others
    p = workloads.small_plain(seed=4, N=1200, d=6, R=16)
    pl = _plan(p, dev, batch_min_rhs=1)
    yb = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    for r in (0, 5, 8, 15):
        ya = pl.matvec(to_dev(p.v[:, r:r + 1], dev)).cpu().numpy()[:, 0]
        assert np.array_equal(ya, yb[:, r])
    yb2 = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    assert np.array_equal(yb, yb2)


def test_degenerate_inputs(dev):
    import paper_2312_00538_amd as lib
    X = np.array([[0.1, -0.2, 0.05, 0.0]])
    pl = lib.Plan(to_dev(X, dev), workloads.consecutive_windows(4), 1.0, precision=FP64)
    y = pl.matvec(to_dev(np.array([[2.0, -1.0, 0.5]]), dev)).cpu().numpy()
    assert np.allclose(y[0], 2.0 * np.array([2.0, -1.0, 0.5]), rtol=TOL_FP64)
    Xs = np.tile(np.array([[0.2, 0.1, -0.1, 0.05, 0.0, 0.3]]), (50, 1))
    v = np.random.default_rng(0).standard_normal((50, 4))
    pl = lib.Plan(to_dev(Xs, dev), workloads.consecutive_windows(6), 0.5, precision=FP64)
    y = pl.matvec(to_dev(v, dev)).cpu().numpy()
    for r in range(4):
        assert rel_l2(y[:, r], np.full(50, 2 * v[:, r].sum())) <= TOL_FP64


def test_full_size_matvec_scaling_sampled(dev):
    # N = 100000, d = 30, 10 windows, 16 right-hand sides: the benchmark's launch shape
    p = workloads.matvec_scaling(seed=0, N=100_000, R=16)
    pl = _plan(p, dev)
    y = pl.matvec(to_dev(p.v, dev)).cpu().numpy()
    rows = np.random.default_rng(11).choice(p.X.shape[0], 96, replace=False)
    ref = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v, rows=rows)
    errs = [rel_l2(y[rows, r], ref[:, r]) for r in range(16)]
    print("full-size FP64 batched rel_l2 per rhs on 96 sampled rows", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL_FP64
