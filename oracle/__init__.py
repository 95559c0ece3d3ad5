"""ORACLE — test infrastructure only.

Plain, slow, obviously-correct CPU FP64 implementations of what the GPU library
computes. Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg
of `bench.py` may import this package; the product library never does, and the
two share no code (the seeded input generators in `workloads.py` are the only
common module and hold none of the method's arithmetic).

Contents, each following the paper (arXiv 2312.00538):
  * anova_matvec / anova_columns / anova_dense — the ANOVA Gaussian kernel
    (Section 3), by direct summation (C, `anova_direct.c`) or dense numpy;
    anova_cross — the same sum from source points to other target points.
  * ipm_dense — the interior point method of Algorithm 1 (Section 2) with the
    Newton system (Section 2, equation "Newton") solved densely.
  * pivoted_cholesky — Algorithm 2 (Section 4) on the dense matrix;
    rp_cholesky — its randomly pivoted variant (Section 4) with given draws.
  * rff_features — random Fourier features of the ANOVA sum (Section 4).
  * nystrom — the Nystrom approximation (Section 4) with LDL^T and clamping.
  * woodbury_apply — the Sherman-Morrison-Woodbury form of the (1,1)-block
    preconditioner (Section 5).
  * saddle_preconditioners — the block-triangular preconditioner of Section 5
    and its block-diagonal SPD analogue; block_triangular_apply — its inverse
    by forward substitution; gmres — right-preconditioned GMRES (Section 5).
  * objectives — dual objective (eq. "kernelsvm"), hinge-loss primal and the
    relative duality gap used as the stopping measure.
  * mi_windows — windows of features by mutual-information ranking (Section 3).
Readings where the paper is silent are listed in the design notes and repeated
in the docstrings below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle_direct.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C direct-sum oracle with gcc (-O2 -fopenmp, no fast-math)."""
    src = os.path.join(_HERE, "anova_direct.c")
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(src):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.oracle_anova_direct.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int32,
                                                P, P, P, ctypes.c_int32, P, ctypes.c_int64, P]
            lib.oracle_anova_direct.restype = ctypes.c_int
            lib.oracle_anova_columns.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int32,
                                                 P, P, P, ctypes.c_int64, P]
            lib.oracle_anova_columns.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(X, windows, sigma, eta):
    X = np.ascontiguousarray(X, dtype=np.float64)
    win = np.ascontiguousarray(windows, dtype=np.int32).reshape(-1, 3)
    P = win.shape[0]
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float64), (P,)))
    et = np.ones(P) if eta is None else np.ascontiguousarray(np.broadcast_to(np.asarray(eta, np.float64), (P,)))
    return X, win, sig, et


def anova_matvec(X, windows, sigma, v, eta=None, rows=None, threads: int | None = None):
    """y = sum_l eta_l K_l v by direct summation (Section 3). v: N or N x R.
    rows: optional target subset; returns len(rows) x R (or N x R)."""
    X, win, sig, et = _prep(X, windows, sigma, eta)
    N, d = X.shape
    v = np.asarray(v, dtype=np.float64)
    vec = v.ndim == 1
    V = np.asfortranarray(v.reshape(N, -1))
    R = V.shape[1]
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rows.shape[0]
    else:
        nr = N
    Y = np.zeros((nr, R), order="F")
    lib = _load()
    old = os.environ.get("OMP_NUM_THREADS")
    rc = lib.oracle_anova_direct(_ptr(X), N, d, _ptr(win), win.shape[0], _ptr(sig), _ptr(et),
                                 _ptr(V), R, _ptr(rows) if rows is not None else None, nr, _ptr(Y))
    if rc != 0:
        raise ValueError("oracle_anova_direct failed")
    return Y[:, 0] if vec else Y


def anova_columns(X, windows, sigma, cols, eta=None):
    """Kernel columns K[:, cols] (Section 3 definition), N x len(cols)."""
    X, win, sig, et = _prep(X, windows, sigma, eta)
    N, d = X.shape
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros((N, cols.shape[0]), order="F")
    _load().oracle_anova_columns(_ptr(X), N, d, _ptr(win), win.shape[0], _ptr(sig), _ptr(et),
                                 _ptr(cols), cols.shape[0], _ptr(out))
    return out


def anova_dense(X, windows, sigma, eta=None):
    """Dense K = sum_l eta_l K_l with (K_l)_{ij} = exp(-sum_{a in W_l}(X_ia - X_ja)^2 / sigma_l^2)
    (Section 3). Numpy, explicit differences, row blocks to bound memory."""
    X, win, sig, et = _prep(X, windows, sigma, eta)
    N = X.shape[0]
    K = np.zeros((N, N))
    blk = max(1, int(2e7 // max(N, 1)))
    for l in range(win.shape[0]):
        f = [int(c) for c in win[l] if c >= 0]
        Xw = X[:, f]
        for s in range(0, N, blk):
            diff = Xw[s:s + blk, None, :] - Xw[None, :, :]
            K[s:s + blk] += et[l] * np.exp(-(diff * diff).sum(-1) / sig[l] ** 2)
    return K


def anova_cross(Xt, Xs, windows, sigma, v, eta=None):
    """y_j = sum_l eta_l sum_i exp(-sum_{a in W_l}(Xt_ja - Xs_ia)^2 / sigma_l^2) v_i for
    targets Xt (M x d) and sources Xs (N x d): the kernel of Section 3 between two
    point sets (the decision function of Section 2 evaluates it at new points).
    Numpy, explicit differences, target blocks to bound memory."""
    Xs, win, sig, et = _prep(Xs, windows, sigma, eta)
    Xt = np.ascontiguousarray(np.asarray(Xt, dtype=np.float64))
    v = np.asarray(v, dtype=np.float64)
    M, N = Xt.shape[0], Xs.shape[0]
    y = np.zeros(M)
    blk = max(1, int(2e7 // max(N, 1)))
    for l in range(win.shape[0]):
        f = [int(c) for c in win[l] if c >= 0]
        for s in range(0, M, blk):
            diff = Xt[s:s + blk, None, f] - Xs[None, :, f]
            y[s:s + blk] += et[l] * (np.exp(-(diff * diff).sum(-1) / sig[l] ** 2) @ v)
    return y


# ----------------------------------------------------------------------------- objectives

def dual_objective(K, y, alpha):
    """e^T alpha - 1/2 alpha^T Y K Y alpha (eq. "kernelsvm")."""
    ya = y * alpha
    return float(alpha.sum() - 0.5 * ya @ (K @ ya))


def objectives_from_kya(kya, y, alpha, lam, C):
    """Dual D, hinge primal Pr and relative gap G = (Pr - D)/(1 + |Pr|), from the
    product K (Y alpha). Decision values f = K Y alpha - lambda (bias b = -lambda,
    which follows from the optimality conditions of Section 2)."""
    quad = float((y * alpha) @ kya)
    D = float(alpha.sum()) - 0.5 * quad
    f = kya - lam
    hinge = np.maximum(0.0, 1.0 - y * f).sum()
    Pr = 0.5 * quad + C * float(hinge)
    return D, Pr, (Pr - D) / (1.0 + abs(Pr))


# ----------------------------------------------------------------------------- IPM (Algorithm 1)

def initial_point(y, C):
    """alpha^0_i = C(2 + y_i)/4 if sum(y) >= 0 else C(2 - y_i)/4, lambda^0 = 0, so
    that xi_alpha^0 = y^T alpha^0 != 0 as Algorithm 1 requires."""
    if y.sum() >= 0:
        a = C * (2.0 + y) / 4.0
    else:
        a = C * (2.0 - y) / 4.0
    return a, 0.0


def ipm_dense(K, y, C, tol=1e-6, tol_inf=1e-1, max_ip=100, sigma_bar=0.6, gamma0=0.99995,
              mu0=1.0, mu_rule="adaptive", record=False, mu_floor=1e-2):
    """Algorithm 1 (Section 2) with the Newton system (eq. "Newton") solved by a
    dense LU solve of the (N+1) x (N+1) saddle-point matrix.

    Per iteration: mu <- sigma_it * mu; Theta = mu (1/alpha^2 + 1/(C-alpha)^2);
    solve [[YKY + Theta, -y], [-y^T, 0]] [da; dl] =
          [e - YKY alpha + lambda y + mu/alpha - mu/(C-alpha); y^T alpha];
    step s = gamma0 * min(1, s_max) with s_max the largest step keeping
    0 < alpha < C (the same step for lambda); update; recompute the
    infeasibilities xi_alpha = y^T alpha and xi_lambda (the first Newton block
    residual at the current mu) and the relative duality gap G.
    Stop when mu <= tol, |xi_alpha|/|xi_alpha^0| <= tol, G <= tol and
    ||xi_lambda||/||xi_lambda^0|| <= tol_inf, or after max_ip steps. The
    xi_lambda ratio keeps the IPM tolerance of Table 1 (1e-1): with a primal
    barrier Newton step the residual of the barrier terms at active bounds does
    not vanish as mu -> 0, so that ratio levels off well above 1e-6.

    Barrier reduction (Section 2 allows a constant factor or one that changes
    every iteration): mu_rule="constant" uses sigma_it = sigma_bar;
    mu_rule="adaptive" uses sigma_it = 1 - (1 - sigma_bar) * s_prev with s_prev
    the previous step length (s_prev = 1 before the first step), i.e. sigma_bar
    after full steps and little reduction after steps cut short by the box.
    Either way mu is not reduced below mu_floor * tol * (1 + |Pr|) / (2 N), the
    value whose central point (duality gap 2 N mu) has the relative gap
    mu_floor * tol: a smaller mu changes nothing the stop test can see, while
    the barrier weights mu / alpha^2 of the rows at a bound grow like 1 / mu.
    Pr is the primal objective of the current iterate.
    """
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    YKY = y[:, None] * K * y[None, :]
    alpha, lam = initial_point(y, C)
    mu = mu0

    def xi_lambda(a, l, m):
        return 1.0 - YKY @ a + l * y + m / a - m / (C - a)

    xa0 = abs(float(y @ alpha))
    xl0 = float(np.linalg.norm(xi_lambda(alpha, lam, mu)))
    xa, xl = xa0, xl0
    kya = K @ (y * alpha)
    D, Pr, G = objectives_from_kya(kya, y, alpha, lam, C)
    it = 0
    hist = []
    s_prev = 1.0
    while it < max_ip:
        if mu <= tol and xa / xa0 <= tol and xl / xl0 <= tol_inf and G <= tol:
            break
        if mu_rule == "constant":
            mu = sigma_bar * mu
        else:
            mu = (1.0 - (1.0 - sigma_bar) * s_prev) * mu
        mu = max(mu, mu_floor * tol * (1.0 + abs(Pr)) / (2.0 * N))
        theta = mu * (1.0 / alpha ** 2 + 1.0 / (C - alpha) ** 2)
        r1 = 1.0 - YKY @ alpha + lam * y + mu / alpha - mu / (C - alpha)
        r2 = float(y @ alpha)
        A = np.zeros((N + 1, N + 1))
        A[:N, :N] = YKY + np.diag(theta)
        A[:N, N] = -y
        A[N, :N] = -y
        sol = np.linalg.solve(A, np.concatenate([r1, [r2]]))
        da, dl = sol[:N], sol[N]
        smax = np.inf
        neg = da < 0
        pos = da > 0
        if neg.any():
            smax = min(smax, float(np.min(-alpha[neg] / da[neg])))
        if pos.any():
            smax = min(smax, float(np.min((C - alpha[pos]) / da[pos])))
        s = gamma0 * min(1.0, smax)
        s_prev = s
        alpha = alpha + s * da
        lam = lam + s * dl
        xa = abs(float(y @ alpha))
        xl = float(np.linalg.norm(xi_lambda(alpha, lam, mu)))
        kya = K @ (y * alpha)
        D, Pr, G = objectives_from_kya(kya, y, alpha, lam, C)
        it += 1
        if record:
            hist.append(dict(it=it, mu=mu, step=s, xa=xa / xa0, xl=xl / xl0, D=D, G=G))
    converged = mu <= tol and xa / xa0 <= tol and xl / xl0 <= tol_inf and G <= tol
    return dict(alpha=alpha, lam=lam, mu=mu, it=it, D=D, Pr=Pr, G=G,
                xa_rel=xa / xa0, xl_rel=xl / xl0, converged=converged, hist=hist)


# ----------------------------------------------------------------------------- Algorithm 2

def rp_cholesky(K, u, err_tol=0.0):
    """Randomly pivoted Cholesky: Algorithm 2 (Section 4) with the pivot of step j
    drawn with probability proportional to the residual diagonal, the variant
    Section 4 cites beside the greedy rule. With the clamped residual diagonal
    d+ = max(d, 0), its running sums C and total T, step j takes the smallest i
    with C_i > u[j] * T. The column of the pivot p is K[:, p] - L L[p]^T over the
    steps so far, scaled by 1 / sqrt(K_pp - |L[p]|^2); then d -= column^2 and
    d_p = 0. Stops when T = 0, when T <= err_tol * trace(K), or when the pivot
    value is not positive. Returns (L, piv) with L N x r in the original row
    order and the pivots in the order chosen."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    u = np.asarray(u, dtype=np.float64)
    L = np.zeros((n, len(u)))
    d = np.diag(K).copy()
    trace0 = float(d.sum())
    piv = []
    for j in range(len(u)):
        dp = np.maximum(d, 0.0)
        total = float(dp.sum())
        if not total > 0.0:
            break
        if err_tol > 0.0 and total <= err_tol * trace0:
            break
        p = int(np.argmax(np.cumsum(dp) > u[j] * total))
        pivval = K[p, p] - float(L[p, :j] @ L[p, :j])
        if not (d[p] > 0.0 and pivval > 0.0):
            break
        col = (K[:, p] - L[:, :j] @ L[p, :j]) / np.sqrt(pivval)
        L[:, j] = col
        d = d - col * col
        d[p] = 0.0
        piv.append(p)
    return L[:, :len(piv)], np.array(piv, dtype=np.int64)


def rff_counts(k, P):
    """Features per window: k // P each, the first k % P windows one more."""
    return [k // P + (1 if l < k % P else 0) for l in range(P)]


def rff_features(X, windows, sigma, w, b, eta=None):
    """Random Fourier features (Section 4) of the ANOVA kernel sum: Z (N x k) with
    the rank split over the windows (rff_counts). Feature j of window l is
    sqrt(eta_l * 2 / k_l) cos(w_j . x^{W_l} + b_j), w_j holding one frequency per
    feature of the window in order (w is k x 3, entries past the window's size
    unused). For w_j ~ N(0, (2 / sigma_l^2) I) and b_j ~ U(0, 2 pi), E[Z Z^T] = K
    (Bochner's theorem for the Gaussian of each window)."""
    X, win, sig, et = _prep(X, windows, sigma, eta)
    w = np.asarray(w, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    k = b.shape[0]
    Z = np.zeros((X.shape[0], k))
    j = 0
    for l, cl in enumerate(rff_counts(k, win.shape[0])):
        f = [int(c) for c in win[l] if c >= 0]
        for _ in range(cl):
            Z[:, j] = np.sqrt(et[l] * 2.0 / cl) * np.cos(X[:, f] @ w[j, :len(f)] + b[j])
            j += 1
    return Z


def pivoted_cholesky(K, k, err_tol=0.0):
    """Greedy pivoted Cholesky of rank <= k (Algorithm 2, Section 4) on a copy of
    the dense K: at step j pick the largest remaining diagonal entry (lowest
    index on ties), swap it to position j symmetrically, take the square root,
    scale the column below and apply the rank-1 update to the trailing block.
    Stops when r = k, the largest remaining diagonal is <= 0, or the remaining
    trace is <= err_tol * trace(K).
    Returns (L, piv) with L N x r in the ORIGINAL row order, K ~= L L^T, and the
    pivot indices in the order chosen."""
    A = np.array(K, dtype=np.float64, copy=True)
    n = A.shape[0]
    perm = np.arange(n)
    trace0 = float(np.trace(A))
    r = 0
    for j in range(n):
        dg = np.diag(A)[j:]
        l = j + int(np.argmax(dg))
        if not (A[l, l] > 0 and r < k):
            break
        if err_tol > 0 and float(dg.sum()) <= err_tol * trace0:
            break
        r += 1
        if l != j:
            A[[j, l], :] = A[[l, j], :]
            A[:, [j, l]] = A[:, [l, j]]
            perm[[j, l]] = perm[[l, j]]
        A[j, j] = np.sqrt(A[j, j])
        A[j + 1:, j] /= A[j, j]
        c = A[j + 1:, j]
        A[j + 1:, j + 1:] -= np.outer(c, c)
    Lp = np.tril(A[:, :r])
    L = np.zeros_like(Lp)
    L[perm] = Lp
    return L, perm[:r].copy()


# ----------------------------------------------------------------------------- Nystrom

def ldl_clamped(M, tau):
    """LDL^T of a symmetric matrix without pivoting; a diagonal entry of D that is
    smaller than tau is replaced by tau (the stabilisation described for the
    Nystrom method, Section 4)."""
    n = M.shape[0]
    L = np.eye(n)
    D = np.zeros(n)
    for j in range(n):
        dj = M[j, j] - (L[j, :j] ** 2) @ D[:j]
        if dj < tau:
            dj = tau
        D[j] = dj
        for i in range(j + 1, n):
            L[i, j] = (M[i, j] - (L[i, :j] * L[j, :j]) @ D[:j]) / dj
    return L, D


def nystrom(K, G, tau_rel=1e-12):
    """Randomized Nystrom approximation (Section 4): Q = orth(K G),
    K ~= (KQ)(Q^T K Q)^{-1}(KQ)^T with Q^T K Q = L D L^T (clamped).
    Returns Zt (N x k) with K ~= Zt Zt^T, Zt = (KQ) L^{-T} D^{-1/2}."""
    Yk = K @ G
    Q, _ = np.linalg.qr(Yk)
    B = K @ Q
    Cm = Q.T @ B
    Cm = 0.5 * (Cm + Cm.T)
    tau = tau_rel * float(np.max(np.diag(Cm)))
    L, D = ldl_clamped(Cm, tau)
    W = np.linalg.solve(L, B.T).T          # B L^{-T}
    return W / np.sqrt(D)[None, :]


# ----------------------------------------------------------------------------- Section 5

def woodbury_apply(theta, y, Zt, r):
    """A_hat^{-1} r for A_hat = Theta + Y Z^T Z Y via the Sherman-Morrison-Woodbury
    form of Section 5:
        Theta^{-1} - Theta^{-1} Y Z^T (I_k + Z Y Theta^{-1} Y Z^T)^{-1} Z Y Theta^{-1}.
    Zt is Z^T (N x k)."""
    tinv = 1.0 / theta
    k = Zt.shape[1]
    M = np.eye(k) + Zt.T @ (Zt * (y * tinv * y)[:, None])
    w = Zt.T @ (y * tinv * r)
    t = np.linalg.solve(M, w)
    return tinv * r - tinv * y * (Zt @ t)


def saddle_matrix(K, y, theta):
    """The Newton matrix A of eq. "Newton": [[YKY + Theta, -y], [-y^T, 0]]."""
    N = y.shape[0]
    A = np.zeros((N + 1, N + 1))
    A[:N, :N] = y[:, None] * K * y[None, :] + np.diag(theta)
    A[:N, N] = -y
    A[N, :N] = -y
    return A


def saddle_preconditioners(Ahat, y):
    """Section 5: block-triangular P = [[Ahat, 0], [-y^T, -1]] and the
    block-diagonal SPD analogue P_d = diag(Ahat, y^T Ahat^{-1} y)."""
    N = y.shape[0]
    Pt = np.zeros((N + 1, N + 1))
    Pt[:N, :N] = Ahat
    Pt[N, :N] = -y
    Pt[N, N] = -1.0
    Pd = np.zeros((N + 1, N + 1))
    Pd[:N, :N] = Ahat
    Pd[N, N] = float(y @ np.linalg.solve(Ahat, y))
    return Pt, Pd


def block_triangular_apply(Ahat, y, g):
    """P^{-1} g for the block-triangular preconditioner of Section 5,
    P = [[Ahat, 0], [-y^T, -1]]: forward substitution by blocks,
    x1 = Ahat^{-1} g1, then -y^T x1 - x2 = g2."""
    N = y.shape[0]
    x1 = np.linalg.solve(Ahat, g[:N])
    return np.concatenate([x1, [-(y @ x1) - g[N]]])


def gmres(A, b, apply_pinv, tol, maxit):
    """GMRES (Saad and Schultz 1986) for A x = b, preconditioned from the right
    (Section 5 pairs GMRES with the non-symmetric P): minimise ||b - A P^{-1} u||
    over the Krylov space of A P^{-1} started at r0 = b, x = P^{-1} u. Arnoldi by
    modified Gram-Schmidt, least squares by Givens rotations; stops when the
    residual estimate |g_{j+1}| <= tol ||b|| or after maxit steps.
    Returns (x, iterations, residual estimates after each step)."""
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n), 0, []
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[:, 0] = b / beta
    hist, j = [], 0
    while j < maxit:
        w = A @ apply_pinv(V[:, j])
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V[:, j + 1] = w / H[j + 1, j]
        for i in range(j):   # earlier rotations on the new column
            a, c = H[i, j], H[i + 1, j]
            H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
        rho = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
        H[j, j], H[j + 1, j] = rho, 0.0
        g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
        j += 1
        hist.append(abs(g[j]))
        if abs(g[j]) <= tol * beta:   # also a breakdown (H[j, j-1] = 0), where g[j] = 0
            break
    u = V[:, :j] @ np.linalg.solve(np.triu(H[:j, :j]), g[:j])
    return apply_pinv(u), j, hist


# ----------------------------------------------------------------------------- windows (Section 3)

def mi_bins(X, bins):
    """Histogram bin of every entry: equal-width bins over each feature's range,
    b = floor((x - min) * (bins / (max - min))) clamped to bins - 1 (all entries
    of a constant feature fall in bin 0)."""
    X = np.asarray(X, dtype=np.float64)
    mn, mx = X.min(axis=0), X.max(axis=0)
    B = np.zeros(X.shape, dtype=np.int64)
    for f in range(X.shape[1]):
        if mx[f] > mn[f]:
            scale = bins / (mx[f] - mn[f])
            B[:, f] = np.minimum(np.floor((X[:, f] - mn[f]) * scale).astype(np.int64), bins - 1)
    return B


def mutual_information(counts):
    """Mutual information (nats) of a joint count table n[b][c] (rows: feature
    bins, columns: classes): sum over n > 0 of (n / N) log(n N / (n_b n_c)),
    bins in order, classes in order."""
    counts = np.asarray(counts, dtype=np.int64)
    Ntot = int(counts.sum())
    nb = counts.sum(axis=1)
    nc = counts.sum(axis=0)
    mi = 0.0
    for b in range(counts.shape[0]):
        for c in range(counts.shape[1]):
            n = int(counts[b, c])
            if n > 0:
                mi += (n / Ntot) * np.log(n * Ntot / (int(nb[b]) * int(nc[c])))
    return mi


def mi_windows(X, labels, bins, P):
    """Windows of features by mutual-information ranking (Section 3 picks the
    windows from the features' mutual information scores): each feature's
    mutual information with the labels is estimated from its histogram
    (mi_bins) against the two classes; features are ranked by it, largest
    first, ties to the lower index; the windows are consecutive triples of the
    ranking, the last one taking the remaining 1 or 2 features when 3P > d.
    Returns (windows P x 3 int32 padded with -1, mi per feature, counts d x bins x 2)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(labels)
    N, d = X.shape
    B = mi_bins(X, bins)
    cls = (y > 0).astype(np.int64)            # class 0: -1, class 1: +1
    counts = np.zeros((d, bins, 2), dtype=np.int64)
    for f in range(d):
        np.add.at(counts[f], (B[:, f], cls), 1)
    mi = np.array([mutual_information(counts[f]) for f in range(d)])
    rank = sorted(range(d), key=lambda f: (-mi[f], f))
    W = np.full((P, 3), -1, dtype=np.int32)
    for l in range(P):
        feats = rank[3 * l: min(d, 3 * l + 3)]
        W[l, :len(feats)] = feats
    return W, mi, counts
