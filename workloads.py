"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only draws random numbers and prepares data matrices (z-score per
column, then scaling into [-1/4, 1/4] as in the paper's preprocessing, Section 6).
It contains none of the method's arithmetic (no kernel, no NFFT, no solver).

The paper's datasets (HIGGS, SUSY, cod-rna; Section 6) are not available; these
generators stand in for them with the same shapes: d = 9 / 20 / 30 features
grouped into windows of at most three consecutive features (Section 3).
All draws use numpy's PCG64 (`numpy.random.default_rng(seed)`) in a fixed order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def consecutive_windows(d: int, width: int = 3) -> np.ndarray:
    """Windows {0,1,2}, {3,4,5}, ...; the last window takes the 1 or 2 leftover
    features. Returned as a P x 3 int32 array padded with -1 (P = ceil(d/3))."""
    P = math.ceil(d / width)
    w = np.full((P, 3), -1, dtype=np.int32)
    for l in range(P):
        feats = list(range(l * width, min(d, (l + 1) * width)))
        w[l, : len(feats)] = feats
    return w


def standardize_scale(X: np.ndarray) -> np.ndarray:
    """z-score each column with the population std (ddof=0), then divide each
    column by 4 * max|x| so every feature lies in [-1/4, 1/4]."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    Z = (X - mu) / sd
    mx = np.abs(Z).max(axis=0)
    mx = np.where(mx > 0, mx, 1.0)
    return np.ascontiguousarray(Z / (4.0 * mx))


@dataclass
class Problem:
    X: np.ndarray                 # N x d float64, row-major
    labels: np.ndarray            # N float64 in {-1, +1}
    windows: np.ndarray           # P x 3 int32, -1 padded
    sigma: float
    C: float | None = None
    v: np.ndarray | None = None   # N x R float64 right-hand sides (column-major use: v[:, r])
    meta: dict = field(default_factory=dict)


def small_plain(seed: int = 0, N: int = 2000, d: int = 9, R: int = 1) -> Problem:
    """N(0,1) features; labels sign(x1+x2+x3 + 0.3 eps) from the raw features with
    sign(0)=+1; then standardize+scale; v ~ N(0,1). Windows of 3 consecutive
    features, sigma = 1, C = 1."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, d))
    eps = rng.standard_normal(N)
    s = X[:, 0] + X[:, 1] + X[:, 2] + 0.3 * eps
    labels = np.where(s >= 0, 1.0, -1.0)
    Xs = standardize_scale(X)
    v = rng.standard_normal((N, R))
    return Problem(Xs, labels, consecutive_windows(d), 1.0, 1.0, v,
                   dict(workload="plain-small", N=N, d=d, seed=seed))


def gaussian_mixture(seed: int = 0, N: int = 100_000, d: int = 30, R: int = 1,
                     noise: float = 0.0, sigma: float = 1.0, C: float | None = None,
                     shift: float = 0.5) -> Problem:
    """Two-class Gaussian mixture: labels N/2 of +1 and N - N/2 of -1, then a
    random permutation; X = N(0, I) + shift * y (class means +-shift * e); then,
    if noise > 0, labels at rng.choice(N, floor(noise*N), replace=False) are
    flipped; then standardize+scale; v ~ N(0,1) of shape N x R."""
    rng = np.random.default_rng(seed)
    y0 = np.concatenate([np.ones(N // 2), -np.ones(N - N // 2)])
    y0 = rng.permutation(y0)
    X = rng.standard_normal((N, d)) + shift * y0[:, None]
    labels = y0.copy()
    nflip = int(math.floor(noise * N))
    if nflip > 0:
        idx = rng.choice(N, nflip, replace=False)
        labels[idx] = -labels[idx]
    Xs = standardize_scale(X)
    v = rng.standard_normal((N, R)) if R > 0 else None
    return Problem(Xs, labels, consecutive_windows(d), sigma, C, v,
                   dict(workload="gaussian-mixture", N=N, d=d, seed=seed, noise=noise))


def matvec_scaling(seed: int = 0, N: int = 100_000, R: int = 1) -> Problem:
    """N = 1e5, d = 30 (10 windows of 3), sigma = 1."""
    p = gaussian_mixture(seed, N=N, d=30, R=R, sigma=1.0)
    p.meta["workload"] = "matvec-scaling"
    return p


def full_ipm(seed: int = 0, N: int = 500_000, R: int = 0) -> Problem:
    """N = 5e5, d = 20 (6 windows of 3 + 1 of 2), 10% label noise, sigma = 0.8, C = 10."""
    p = gaussian_mixture(seed, N=N, d=20, R=R, noise=0.10, sigma=0.8, C=10.0)
    p.meta["workload"] = "full-ipm"
    return p


def random_vectors(seed: int, N: int, R: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, R))


def serving_stream(seed: int, n_requests: int, rate: float = 2.0,
                   n_range=(5_000, 1_000_000), d_range=(6, 60),
                   sigma_range=(0.5, 2.0), C_range=(0.1, 100.0)) -> list[dict]:
    """Poisson arrivals (exponential inter-arrival times with mean 1/rate) of SVM
    training requests; per request N log-uniform, d uniform integer, sigma and C
    log-uniform, and a per-request data seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        sigma = float(math.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]))))
        C = float(math.exp(rng.uniform(math.log(C_range[0]), math.log(C_range[1]))))
        out.append(dict(id=i, arrival=t, N=N, d=d, sigma=sigma, C=C, data_seed=int(rng.integers(0, 2**31 - 1))))
    return out


def cv_grid(seed: int = 0, N: int = 50_000, d: int = 15, folds: int = 5,
            n_sigma: int = 8, sigma_range=(0.25, 4.0), n_C: int = 8, C_range=(0.1, 1000.0)) -> dict:
    """Hyperparameter grid over cross-validation folds (a stand-in for the
    paper's parameter search, Section 6.3). Data as gaussian_mixture(seed, N, d)
    (shift 0.5, no noise). Folds: a permutation of the N points (drawn after the
    data, from rng(seed + 1)) cut into `folds` equal holdout blocks; the
    training part of each fold is class balanced by keeping a random subset
    (without replacement, from the same rng) of the majority class of the size
    of the minority class, so training sizes are uneven and at most
    N (folds - 1) / folds. sigma: n_sigma log-spaced values, C: n_C log-spaced
    values. Returns dict(problem, folds=[(train_idx, holdout_idx)], sigmas, Cs)."""
    p = gaussian_mixture(seed, N=N, d=d, R=0)
    rng = np.random.default_rng(seed + 1)
    perm = rng.permutation(N)
    size = N // folds
    out = []
    for f in range(folds):
        hold = np.sort(perm[f * size:(f + 1) * size])
        train = np.sort(np.concatenate([perm[:f * size], perm[(f + 1) * size:]]))
        pos = train[p.labels[train] > 0]
        neg = train[p.labels[train] < 0]
        m = min(len(pos), len(neg))
        if len(pos) > m:
            pos = np.sort(rng.choice(pos, m, replace=False))
        if len(neg) > m:
            neg = np.sort(rng.choice(neg, m, replace=False))
        out.append((np.sort(np.concatenate([pos, neg])), hold))
    sigmas = np.geomspace(sigma_range[0], sigma_range[1], n_sigma)
    Cs = np.geomspace(C_range[0], C_range[1], n_C)
    p.meta["workload"] = "cv-grid"
    return dict(problem=p, folds=out, sigmas=sigmas, Cs=Cs)


def graded_features(seed: int = 0, N: int = 20_000, d: int = 14, order=None) -> Problem:
    """Balanced +-1 labels and d features of graded relevance: feature f is
    s_f * y + N(0, 1) with s_f = 2 (1 - rank_f / d), rank_f = order[f] (a
    permutation of 0..d-1; the identity if None), so that feature order[f] = 0
    carries the label most strongly and the last rank not at all; then
    standardize+scale. Windows: consecutive, sigma = 1. The informative order
    is stored in meta["order"]."""
    rng = np.random.default_rng(seed)
    y = np.where(np.arange(N) < N // 2, 1.0, -1.0)
    y = y[rng.permutation(N)]
    order = np.arange(d) if order is None else np.asarray(order)
    s = 2.0 * (1.0 - order / d)
    X = s[None, :] * y[:, None] + rng.standard_normal((N, d))
    X = standardize_scale(X)
    p = Problem(X=X, labels=y, windows=consecutive_windows(d), sigma=1.0)
    p.meta["workload"] = "graded-features"
    p.meta["order"] = order
    return p
