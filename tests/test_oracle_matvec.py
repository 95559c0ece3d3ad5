"""Pins for the oracle's ANOVA kernel sum (Section 3, extended Gaussian ANOVA kernel).

Each check ties the oracle to something other than itself: a library routine
(scikit-learn's RBF kernel), closed forms for tiny inputs, and invariants of the
kernel (symmetry, unit diagonal, positive semi-definiteness, translation and
scale invariance, Hadamard-product structure)."""
import numpy as np
import pytest
from sklearn.metrics.pairwise import rbf_kernel

import oracle
import workloads


def _rand(N=60, d=7, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.25, 0.25, size=(N, d))
    return X, rng.standard_normal(N)


def test_direct_sum_matches_sklearn_rbf_per_window():
    X, v = _rand(80, 8)
    win = workloads.consecutive_windows(8)          # {0,1,2},{3,4,5},{6,7}
    sig = np.array([0.3, 0.7, 1.1])
    eta = np.array([1.0, 0.5, 2.0])
    y = oracle.anova_matvec(X, win, sig, v, eta=eta)
    ref = np.zeros(80)
    for l in range(3):
        f = [c for c in win[l] if c >= 0]
        ref += eta[l] * rbf_kernel(X[:, f], gamma=1.0 / sig[l] ** 2) @ v
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_dense_matches_direct_sum():
    X, v = _rand(120, 9, seed=3)
    win = workloads.consecutive_windows(9)
    K = oracle.anova_dense(X, win, 0.5)
    assert np.allclose(K @ v, oracle.anova_matvec(X, win, 0.5, v), rtol=1e-12, atol=1e-11)


def test_multiple_rhs_and_row_subset():
    X, _ = _rand(50, 6, seed=4)
    win = workloads.consecutive_windows(6)
    V = np.random.default_rng(5).standard_normal((50, 3))
    Y = oracle.anova_matvec(X, win, 0.4, V)
    for r in range(3):
        assert np.allclose(Y[:, r], oracle.anova_matvec(X, win, 0.4, V[:, r]), rtol=1e-14, atol=1e-14)
    rows = np.array([7, 0, 49])
    assert np.allclose(oracle.anova_matvec(X, win, 0.4, V, rows=rows), Y[rows], rtol=1e-14, atol=1e-14)


def test_single_point_gives_sum_of_weights():
    X = np.array([[0.1, -0.2, 0.05, 0.2]])
    win = workloads.consecutive_windows(4)
    eta = np.array([0.7, 1.9])
    y = oracle.anova_matvec(X, win, [0.3, 2.0], np.array([2.5]), eta=eta)
    assert y[0] == pytest.approx(2.5 * eta.sum(), rel=1e-15)


def test_identical_points():
    X = np.tile(np.array([[0.1, -0.2, 0.05, 0.2, 0.0, 0.1]]), (10, 1))
    v = np.arange(10.0)
    y = oracle.anova_matvec(X, workloads.consecutive_windows(6), 0.3, v)
    assert np.allclose(y, 2 * v.sum(), rtol=1e-15)


def test_two_points_closed_form():
    X = np.array([[0.05], [0.2]])
    v = np.array([1.3, -0.4])
    sig = 0.11
    y = oracle.anova_matvec(X, np.array([[0, -1, -1]]), sig, v)
    k = np.exp(-(0.15 ** 2) / sig ** 2)
    assert np.allclose(y, [v[0] + k * v[1], v[1] + k * v[0]], rtol=1e-15)


def test_two_points_three_features_closed_form():
    X = np.array([[0.0, 0.1, -0.1], [0.05, -0.1, 0.2]])
    v = np.array([0.5, 2.0])
    sig = 0.4
    y = oracle.anova_matvec(X, np.array([[0, 1, 2]]), sig, v)
    r2 = 0.05 ** 2 + 0.2 ** 2 + 0.3 ** 2
    k = np.exp(-r2 / sig ** 2)
    assert np.allclose(y, [v[0] + k * v[1], v[1] + k * v[0]], rtol=1e-15)


def test_large_sigma_and_far_points_limits():
    X, v = _rand(30, 6, seed=7)
    win = workloads.consecutive_windows(6)
    y = oracle.anova_matvec(X, win, 1e6, v)
    assert np.allclose(y, 2 * v.sum(), rtol=1e-9)
    Xf = np.arange(30.0)[:, None] * np.ones((1, 6))
    y = oracle.anova_matvec(Xf, win, 0.05, v)
    assert np.allclose(y, 2 * v, rtol=1e-14)


def test_symmetry_unit_diagonal_psd():
    X, _ = _rand(70, 9, seed=8)
    win = workloads.consecutive_windows(9)
    K = oracle.anova_dense(X, win, 0.6)
    assert np.allclose(K, K.T, atol=0)
    assert np.allclose(np.diag(K), 3.0, rtol=1e-15)
    assert np.linalg.eigvalsh(K).min() > -1e-12
    rng = np.random.default_rng(9)
    u, w = rng.standard_normal(70), rng.standard_normal(70)
    Ku = oracle.anova_matvec(X, win, 0.6, u)
    Kw = oracle.anova_matvec(X, win, 0.6, w)
    assert u @ Kw == pytest.approx(w @ Ku, rel=1e-12)


def test_translation_scaling_and_permutation_invariance():
    X, v = _rand(40, 6, seed=10)
    win = workloads.consecutive_windows(6)
    y = oracle.anova_matvec(X, win, 0.3, v)
    assert np.allclose(oracle.anova_matvec(X + 0.37, win, 0.3, v), y, rtol=1e-12)
    assert np.allclose(oracle.anova_matvec(3.0 * X, win, 0.9, v), y, rtol=1e-12)
    assert np.allclose(oracle.anova_matvec(X, win[::-1].copy(), 0.3, v), y, rtol=1e-12)
    wp = win[:, [2, 0, 1]].copy()
    assert np.allclose(oracle.anova_matvec(X, wp, 0.3, v), y, rtol=1e-12)


def test_window_kernel_is_hadamard_product_of_1d_kernels():
    X, _ = _rand(25, 3, seed=11)
    K3 = oracle.anova_dense(X, np.array([[0, 1, 2]]), 0.35)
    K1 = [oracle.anova_dense(X, np.array([[a, -1, -1]]), 0.35) for a in range(3)]
    assert np.allclose(K3, K1[0] * K1[1] * K1[2], rtol=1e-13)
    cols = oracle.anova_columns(X, np.array([[0, 1, 2]]), 0.35, [3, 17])
    assert np.allclose(cols, K3[:, [3, 17]], rtol=1e-13)


def test_feature_choice_matters():
    # a window that reads the wrong feature must change the result
    X, v = _rand(30, 4, seed=12)
    a = oracle.anova_matvec(X, np.array([[0, 1, -1]]), 0.2, v)
    b = oracle.anova_matvec(X, np.array([[0, 2, -1]]), 0.2, v)
    assert np.abs(a - b).max() > 1e-3


def test_cross_kernel_on_the_same_points_is_the_direct_sum():
    # targets = sources: the two-set sum equals the C direct sum of the same matvec
    p = workloads.small_plain(seed=4, N=300)
    y2 = oracle.anova_cross(p.X, p.X, p.windows, p.sigma, p.v[:, 0])
    y1 = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v[:, 0]).reshape(-1)
    assert np.allclose(y2, y1, rtol=1e-12, atol=1e-12)


def test_cross_kernel_closed_forms():
    # a target on a source point with a unit coefficient sees every window's
    # K(x, x) = 1: the value is the sum of eta; a far target sees nothing
    p = workloads.small_plain(seed=5, N=50)
    e = np.zeros(50)
    e[7] = 1.0
    eta = np.array([1.0, 2.0, 0.5])
    y = oracle.anova_cross(p.X[[7]], p.X, p.windows, p.sigma, e, eta=eta)
    assert np.isclose(y[0], eta.sum(), rtol=0, atol=1e-15)
    far = p.X[[7]] + 100.0
    assert oracle.anova_cross(far, p.X, p.windows, p.sigma, np.ones(50))[0] == 0.0
