"""GPU parity of the window selection by mutual-information ranking
(Section 3) against the oracle: the same windows, and the same estimates to
1e-12 (both sides bin in FP64 with the same expression, so the integer
histograms agree exactly; a count off by one would move an estimate by ~1e-5)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _both(p, dev, bins, P):
    import paper_2312_00538_amd as lib
    W, mi = lib.mi_windows(to_dev(p.X, dev), to_dev(p.labels, dev), bins=bins, P=P)
    Wo, mio, _ = oracle.mi_windows(p.X, p.labels, bins, P)
    return W, mi, Wo, mio


@pytest.mark.parametrize("N,d,bins,P,seed", [(20000, 14, 32, 5, 1), (777, 8, 2, 3, 2), (5001, 20, 1024, 4, 3),
                                             (100_000, 30, 32, 10, 4)])
def test_windows_and_estimates_match_the_oracle(dev, N, d, bins, P, seed):
    order = np.random.default_rng(seed).permutation(d)
    p = workloads.graded_features(seed=seed, N=N, d=d, order=order)
    W, mi, Wo, mio = _both(p, dev, bins, P)
    print(f"N={N} d={d} bins={bins} P={P} windows={W.tolist()} max rel diff={np.max(np.abs(mi - mio) / np.maximum(mio, 1e-300)):.2e}")
    assert W.tolist() == Wo.tolist()
    assert np.allclose(mi, mio, rtol=1e-12, atol=1e-15)


def test_degenerate_inputs(dev):
    # one row (every feature constant: all estimates 0, index order); a constant
    # column among informative ones; identical columns (ties to the lower index)
    p = workloads.graded_features(seed=5, N=1, d=4)
    W, mi, Wo, mio = _both(p, dev, 8, 2)
    assert W.tolist() == Wo.tolist() == [[0, 1, 2], [3, -1, -1]]
    assert np.all(mi == 0.0)
    q = workloads.graded_features(seed=6, N=3000, d=3)
    X = np.concatenate([q.X[:, [2]], np.full((3000, 1), 0.125), q.X, q.X[:, [2]]], axis=1)
    r = workloads.Problem(X=np.ascontiguousarray(X), labels=q.labels, windows=q.windows, sigma=1.0)
    W, mi, Wo, mio = _both(r, dev, 16, 2)
    assert W.tolist() == Wo.tolist()
    assert mi[1] == 0.0
    ranked = [f for f in W.reshape(-1) if f >= 0]
    assert ranked.index(0) < ranked.index(4) < ranked.index(5)


def test_selected_windows_drive_a_plan(dev):
    # the windows feed anova_plan_create as they are: the matvec on them meets
    # the 1e-4 bar against the oracle's direct sum on the same windows
    import paper_2312_00538_amd as lib
    p = workloads.graded_features(seed=7, N=3000, d=10, order=np.random.default_rng(7).permutation(10))
    W, _ = lib.mi_windows(to_dev(p.X, dev), to_dev(p.labels, dev), bins=32)
    pl = lib.Plan(to_dev(p.X, dev), W, 1.0)
    v = np.random.default_rng(8).standard_normal(3000)
    y = pl.matvec(to_dev(v, dev)).cpu().numpy()
    ref = oracle.anova_matvec(p.X, W, 1.0, v)
    print("windows", W.tolist(), "rel_l2", rel_l2(y, ref))
    assert rel_l2(y, ref) <= 1e-4


def test_bad_arguments(dev):
    import paper_2312_00538_amd as lib
    p = workloads.graded_features(seed=9, N=100, d=5)
    X, y = to_dev(p.X, dev), to_dev(p.labels, dev)
    for kw in (dict(bins=1), dict(bins=1025), dict(P=3), dict(P=0)):
        with pytest.raises(lib.AnovaError) as e:
            lib.mi_windows(X, y, **kw)
        assert e.value.status == lib.INVALID_ARG
    Xn = p.X.copy()
    Xn[3, 1] = np.nan
    with pytest.raises(lib.AnovaError):
        lib.mi_windows(to_dev(Xn, dev), y)
