"""Pins for the oracle's interior point method (Algorithm 1, Section 2), its
preconditioner pieces (Algorithm 2 and the Nystrom method of Section 4, the
Woodbury form and the saddle-point preconditioners of Section 5).

The IPM is pinned against brute-force enumeration of active sets (N <= 7), the
two-point closed form, the diagonal-kernel closed form, scikit-learn's SVC on the
same precomputed kernel (a different algorithm for the same dual QP), and the
KKT conditions at termination."""
import itertools
import json
import os

import numpy as np
import pytest
from sklearn.svm import SVC

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _dual(K, y, a):
    return oracle.dual_objective(K, y, a)


def brute_force_svm(K, y, C):
    """Exact optimum of the dual QP by enumerating every assignment of each
    alpha_i to {0, C, free} and solving the equality-constrained stationarity
    system [YKY_FF, -y_F; -y_F^T, 0] for the free block."""
    N = len(y)
    Q = y[:, None] * K * y[None, :]
    best = -np.inf
    best_a = None
    for assign in itertools.product((0, 1, 2), repeat=N):
        a = np.zeros(N)
        F = [i for i in range(N) if assign[i] == 2]
        U = [i for i in range(N) if assign[i] == 1]
        a[U] = C
        if F:
            nf = len(F)
            A = np.zeros((nf + 1, nf + 1))
            A[:nf, :nf] = Q[np.ix_(F, F)]
            A[:nf, nf] = -y[F]
            A[nf, :nf] = -y[F]
            rhs = np.concatenate([1.0 - Q[np.ix_(F, U)] @ a[U], [y[U] @ a[U]]])
            try:
                sol = np.linalg.solve(A, rhs)
            except np.linalg.LinAlgError:
                continue
            a[F] = sol[:nf]
        if abs(y @ a) > 1e-9 or (a < -1e-12).any() or (a > C + 1e-12).any():
            continue
        val = _dual(K, y, a)
        if val > best:
            best, best_a = val, a.copy()
    return best, best_a


@pytest.mark.parametrize("seed,N,C", [(0, 5, 1.0), (1, 6, 0.5), (2, 7, 3.0)])
def test_ipm_matches_brute_force(seed, N, C):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.25, 0.25, (N, 4))
    y = np.where(rng.standard_normal(N) > 0, 1.0, -1.0)
    y[0], y[1] = 1.0, -1.0
    K = oracle.anova_dense(X, workloads.consecutive_windows(4), 0.15)
    best, _ = brute_force_svm(K, y, C)
    r = oracle.ipm_dense(K, y, C)
    assert r["converged"]
    assert r["D"] == pytest.approx(best, rel=1e-6, abs=1e-9)


def test_two_point_closed_form():
    X = np.array([[0.0, 0.1, 0.0], [0.1, -0.05, 0.2]])
    y = np.array([1.0, -1.0])
    K = oracle.anova_dense(X, np.array([[0, 1, 2]]), 0.3)
    k0, k = K[0, 0], K[0, 1]
    for C in (100.0, 0.3):
        a = min(C, 1.0 / (k0 - k))
        r = oracle.ipm_dense(K, y, C)
        assert r["converged"]
        # at an active bound the interior iterate stays O(mu) inside the box
        assert np.allclose(r["alpha"], a, rtol=1e-6, atol=0.0 if a < C else 10 * r["mu"] / 1e-2)
        if a < C:
            assert r["lam"] == pytest.approx(0.0, abs=1e-6)
            assert r["D"] == pytest.approx(1.0 / (k0 - k), rel=1e-6)


def test_diagonal_kernel_closed_form():
    # points far apart relative to sigma: K = P * I, so alpha_i = (1 + lam y_i)/P
    N, P = 9, 2
    X = np.arange(N, dtype=float)[:, None] * np.ones((1, 6))
    y = np.array([1, 1, 1, 1, 1, -1, -1, -1, -1], dtype=float)
    K = oracle.anova_dense(X, np.array([[0, 1, 2], [3, 4, 5]]), 0.01)
    assert np.allclose(K, P * np.eye(N))
    lam = -y.sum() / N
    r = oracle.ipm_dense(K, y, 10.0)
    assert r["converged"]
    assert np.allclose(r["alpha"], (1.0 + lam * y) / P, rtol=1e-6)
    assert r["lam"] == pytest.approx(lam, rel=1e-5)


def test_ipm_agrees_with_sklearn_svc_dual():
    p = workloads.small_plain(seed=3, N=300)
    K = oracle.anova_dense(p.X, p.windows, p.sigma)
    r = oracle.ipm_dense(K, p.labels, 1.0)
    assert r["converged"]
    svc = SVC(C=1.0, kernel="precomputed", tol=1e-10, max_iter=-1).fit(K, p.labels)
    a = np.zeros(300)
    a[svc.support_] = np.abs(svc.dual_coef_[0])
    d_svc = _dual(K, p.labels, a)
    assert r["D"] == pytest.approx(d_svc, rel=1e-6)
    # decision values agree where the solution is unique (the dual optimum's K Y alpha)
    f_ipm = K @ (p.labels * r["alpha"]) - r["lam"]
    f_svc = svc.decision_function(K)
    assert np.max(np.abs(f_ipm - f_svc)) < 1e-3


def test_kkt_conditions_at_termination():
    p = workloads.small_plain(seed=4, N=250)
    K = oracle.anova_dense(p.X, p.windows, p.sigma)
    C = 1.0
    r = oracle.ipm_dense(K, p.labels, C)
    a, lam, mu = r["alpha"], r["lam"], r["mu"]
    assert r["converged"] and r["G"] <= 1e-6 and r["G"] >= -1e-12
    assert (a > 0).all() and (a < C).all()
    assert abs(p.labels @ a) <= 1e-8 * C * 250
    # complementarity of the barrier pair z = mu/alpha, s = mu/(C - alpha)
    z, s = mu / a, mu / (C - a)
    assert a @ z + (C - a) @ s == pytest.approx(2 * 250 * mu, rel=1e-12)
    # reduced costs: free SVs sit on the margin, bounded ones on the correct side
    f = K @ (p.labels * a) - lam
    m = p.labels * f
    free = (a > 1e-3 * C) & (a < (1 - 1e-3) * C)
    assert np.all(np.abs(m[free] - 1.0) < 1e-2)
    assert np.all(m[a < 1e-6 * C] > 1.0 - 1e-3)
    assert np.all(m[a > (1 - 1e-6) * C] < 1.0 + 1e-3)


def test_weak_duality_for_feasible_points():
    p = workloads.small_plain(seed=5, N=100)
    K = oracle.anova_dense(p.X, p.windows, p.sigma)
    a, _ = oracle.initial_point(p.labels, 1.0)
    # project onto y^T a = 0 by scaling the majority class
    rng = np.random.default_rng(0)
    for _ in range(5):
        a = rng.uniform(0, 1.0, 100)
        pos, neg = p.labels > 0, p.labels < 0
        a[pos] *= a[neg].sum() / a[pos].sum()
        if (a <= 1.0).all():
            D, Pr, G = oracle.objectives_from_kya(K @ (p.labels * a), p.labels, a, 0.0, 1.0)
            assert Pr - D >= -1e-10


def test_initial_point_has_nonzero_infeasibility():
    for y in (np.array([1.0, -1.0, 1.0, -1.0]), np.array([1.0, 1.0, -1.0]), np.array([-1.0, -1.0, 1.0])):
        a, lam = oracle.initial_point(y, 2.0)
        assert abs(y @ a) > 0 and lam == 0.0
        assert set(np.round(a / 2.0, 12)) <= {0.25, 0.75}


def test_table1_defaults_fixture():
    t = json.load(open(os.path.join(GOLD, "table1_parameters.json")))
    assert t["barrier_reduction"] == 0.6 and t["step_to_boundary"] == 0.99995 and t["mu0"] == 1.0


# ----------------------------------------------------------------------------- Algorithm 2

def test_pivoted_cholesky_full_rank_is_cholesky_of_permuted_matrix():
    rng = np.random.default_rng(1)
    X = rng.uniform(-0.25, 0.25, (30, 3))
    K = oracle.anova_dense(X, np.array([[0, 1, 2]]), 0.05)
    L, piv = oracle.pivoted_cholesky(K, 30)
    assert len(piv) == 30 and sorted(piv) == list(range(30))
    Lp = L[piv]                     # rows in pivot order: lower triangular
    ref = np.linalg.cholesky(K[np.ix_(piv, piv)])
    assert np.allclose(Lp, ref, rtol=1e-10, atol=1e-12)
    assert piv[0] == 0              # constant diagonal: lowest index wins the tie


def test_pivoted_cholesky_low_rank_is_column_nystrom_on_pivots():
    p = workloads.small_plain(seed=2, N=120)
    K = oracle.anova_dense(p.X, p.windows, 0.2)
    L, piv = oracle.pivoted_cholesky(K, 15)
    approx = K[:, piv] @ np.linalg.solve(K[np.ix_(piv, piv)], K[piv, :])
    assert np.allclose(L @ L.T, approx, atol=1e-9)
    # greedy choice: each pivot had the largest residual diagonal at its step
    res = np.diag(K).copy()
    Lk = np.zeros((120, 0))
    for j, q in enumerate(piv):
        assert res[q] == pytest.approx(res.max(), rel=1e-10)
        Lk = L[:, : j + 1]
        res = np.diag(K) - (Lk ** 2).sum(1)
    tr = [np.trace(K) - (L[:, :j] ** 2).sum() for j in range(16)]
    assert all(tr[j + 1] <= tr[j] + 1e-12 for j in range(15))


def test_pivoted_cholesky_stops_on_error_tolerance():
    p = workloads.small_plain(seed=2, N=200)
    K = oracle.anova_dense(p.X, p.windows, 1.0)
    L, piv = oracle.pivoted_cholesky(K, 200, err_tol=1e-5)
    r = L.shape[1]
    assert r < 200
    assert np.trace(K - L @ L.T) <= 1e-5 * np.trace(K) + 1e-12


# ----------------------------------------------------------------------------- Nystrom

def test_nystrom_full_rank_reproduces_k():
    p = workloads.small_plain(seed=6, N=40)
    K = oracle.anova_dense(p.X, p.windows, 0.05)
    G = np.random.default_rng(0).standard_normal((40, 40))
    Zt = oracle.nystrom(K, G)
    assert np.allclose(Zt @ Zt.T, K, atol=1e-8 * np.abs(K).max())


def test_nystrom_with_permutation_columns_is_column_nystrom():
    p = workloads.small_plain(seed=7, N=50)
    K = oracle.anova_dense(p.X, p.windows, 0.2)
    S = [3, 11, 20, 41, 7]
    G = np.zeros((50, 5))
    G[S, range(5)] = 1.0
    # orth(K G) spans K[:, S]; the Nystrom formula with Q = I[:, S] gives K[:,S] K_SS^{-1} K[S,:]
    Q = np.zeros((50, 5))
    Q[S, range(5)] = 1.0
    KQ = K @ Q
    approx = KQ @ np.linalg.solve(Q.T @ KQ, KQ.T)
    ref = K[:, S] @ np.linalg.solve(K[np.ix_(S, S)], K[S, :])
    assert np.allclose(approx, ref, atol=1e-10)
    # the randomized variant with G = K^{-1}-free columns spans range(K I_S) and
    # gives the best approximation of that subspace: error <= column Nystrom error
    Zt = oracle.nystrom(K, G)
    assert np.linalg.norm(K - Zt @ Zt.T, 2) <= np.linalg.norm(K - ref, 2) * (1 + 1e-8) + 1e-12


def test_ldl_clamp():
    M = np.array([[4.0, 2.0], [2.0, 1.0]])    # singular
    L, D = oracle.ldl_clamped(M, 1e-6)
    assert D[0] == 4.0 and D[1] == 1e-6
    assert L[1, 0] == 0.5


# ----------------------------------------------------------------------------- Section 5

def test_woodbury_equals_dense_inverse():
    rng = np.random.default_rng(3)
    N, k = 60, 8
    Zt = rng.standard_normal((N, k))
    y = np.where(rng.standard_normal(N) > 0, 1.0, -1.0)
    theta = rng.uniform(1e-3, 10, N)
    r = rng.standard_normal(N)
    A = np.diag(theta) + (y[:, None] * Zt) @ (y[:, None] * Zt).T
    assert np.allclose(oracle.woodbury_apply(theta, y, Zt, r), np.linalg.solve(A, r), rtol=1e-9, atol=1e-12)


def test_saddle_point_preconditioner_spectra():
    p = workloads.small_plain(seed=8, N=40)
    K = oracle.anova_dense(p.X, p.windows, 0.3)
    y = p.labels
    theta = np.random.default_rng(1).uniform(0.1, 5.0, 40)
    A = oracle.saddle_matrix(K, y, theta)
    A11 = A[:40, :40]
    Pt, Pd = oracle.saddle_preconditioners(A11, y)
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(Pt, A)).real)
    s = float(y @ np.linalg.solve(A11, y))
    assert np.sum(np.isclose(ev, 1.0, atol=1e-8)) >= 40
    assert np.min(np.abs(ev - s)) < 1e-8 * max(1.0, s)
    evd = np.linalg.eigvals(np.linalg.solve(Pd, A)).real
    targets = np.array([1.0, (1 + 5 ** 0.5) / 2, (1 - 5 ** 0.5) / 2])
    assert np.all(np.min(np.abs(evd[:, None] - targets[None, :]), axis=1) < 1e-8)


def test_rp_cholesky_full_rank_reproduces_k():
    # rank N: every diagonal entry becomes a pivot and L L^T = K whatever the draws
    rng = np.random.default_rng(3)
    A = rng.standard_normal((7, 7))
    K = A @ A.T + 0.1 * np.eye(7)
    u = rng.uniform(size=7)
    L, piv = oracle.rp_cholesky(K, u)
    assert sorted(piv.tolist()) == list(range(7))
    assert np.allclose(L @ L.T, K, atol=1e-12, rtol=1e-12)


def test_rp_cholesky_draws_on_the_identity():
    # K = I: the remaining indices all carry weight 1, so draw u picks the
    # floor(u * m)-th remaining index (0-based) among the m left
    u = np.array([0.95, 0.0, 0.5, 0.34, 0.99, 0.2])
    L, piv = oracle.rp_cholesky(np.eye(6), u)
    left, expect = list(range(6)), []
    for x in u:
        q = left[int(np.floor(x * len(left)))]
        expect.append(q)
        left.remove(q)
    assert piv.tolist() == expect
    assert np.allclose(np.abs(L[piv, range(6)]), 1.0)


def test_rp_cholesky_zero_draw_takes_the_first_positive_diagonal():
    K = np.diag([0.0, 0.0, 2.0, 3.0])
    L, piv = oracle.rp_cholesky(K, [0.0, 0.0])
    assert piv.tolist() == [2, 3]
    assert np.allclose(L[:, 0], [0, 0, np.sqrt(2.0), 0])


def test_rff_zero_draws_give_the_normalisation():
    # w = 0, b = 0: every feature of window l is sqrt(2 eta_l / k_l), so every
    # entry of Z Z^T is sum_l 2 eta_l
    p = workloads.small_plain(seed=2, N=20)
    eta = np.array([1.0, 0.5, 2.0])
    Z = oracle.rff_features(p.X, p.windows, p.sigma, np.zeros((11, 3)), np.zeros(11), eta=eta)
    assert np.allclose(Z @ Z.T, 2.0 * eta.sum(), rtol=1e-14, atol=0)


def test_rff_expectation_is_the_kernel():
    # many features drawn as specified reproduce K (points about sigma apart, so
    # a wrong frequency variance would miss by far more than the tolerance)
    rng = np.random.default_rng(4)
    X = rng.uniform(-0.5, 0.5, size=(25, 6))
    win = workloads.consecutive_windows(6)
    sigma = 0.5
    k = 2 * 40000
    w = rng.standard_normal((k, 3)) * np.sqrt(2.0) / sigma
    b = rng.uniform(0, 2 * np.pi, size=k)
    Z = oracle.rff_features(X, win, sigma, w, b)
    K = oracle.anova_dense(X, win, sigma)
    err = np.abs(Z @ Z.T - K).max()
    print("max |Z Z^T - K|", err)
    assert err < 0.04
    # half the frequency variance misses clearly
    Z2 = oracle.rff_features(X, win, sigma, w / np.sqrt(2.0), b)
    assert np.abs(Z2 @ Z2.T - K).max() > 0.1


def _newton_system(seed, N):
    p = workloads.small_plain(seed=seed, N=N)
    K = oracle.anova_dense(p.X, p.windows, 0.3)
    y = p.labels
    theta = np.random.default_rng(seed + 1).uniform(0.1, 5.0, N)
    A = oracle.saddle_matrix(K, y, theta)
    b = np.random.default_rng(seed + 2).standard_normal(N + 1)
    return A, y, b


def test_block_triangular_apply_inverts_p():
    # P^{-1} applied to P e_j gives e_j back, column by column
    A, y, _ = _newton_system(4, 30)
    Pt, _ = oracle.saddle_preconditioners(A[:30, :30], y)
    back = np.stack([oracle.block_triangular_apply(A[:30, :30], y, Pt[:, j]) for j in range(31)], axis=1)
    assert np.allclose(back, np.eye(31), atol=1e-10)


def test_gmres_without_preconditioner_is_exact_after_n_steps():
    # Krylov space of dimension n: the minimiser is the solution itself
    A, y, b = _newton_system(5, 25)
    x, its, hist = oracle.gmres(A, b, lambda v: v, tol=0.0, maxit=26)
    assert its == 26
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)


def test_gmres_residual_estimates_are_true_residuals_and_decrease():
    A, y, b = _newton_system(6, 40)
    Ahat = A[:40, :40] + np.diag(np.linspace(0.0, 0.5, 40))   # an inexact (1,1) block
    pinv = lambda v: oracle.block_triangular_apply(Ahat, y, v)
    for m in range(1, 6):
        x, its, hist = oracle.gmres(A, b, pinv, tol=0.0, maxit=m)
        assert its == m
        assert np.linalg.norm(b - A @ x) == pytest.approx(hist[-1], rel=1e-8, abs=1e-12)
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))


def test_gmres_with_exact_block_converges_in_two_steps():
    # with Ahat = A the preconditioned matrix has the two eigenvalues 1 and
    # y^T A^{-1} y and a minimal polynomial of degree 2 (Section 5)
    A, y, b = _newton_system(7, 40)
    x, its, hist = oracle.gmres(A, b, lambda v: oracle.block_triangular_apply(A[:40, :40], y, v),
                                tol=1e-12, maxit=10)
    assert its == 2
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
