"""GPU tests of the decision function f(x) = sum_j alpha_j y_j k(x, x_j) - lambda
(Section 2) at points other than the training points: the kernel sum with
targets other than its sources, against the FP64 oracle's two-set direct sum."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def trained(dev):
    import paper_2312_00538_amd as lib
    p = workloads.gaussian_mixture(seed=6, N=1500, d=9, sigma=0.8, C=2.0, R=0)
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    y = to_dev(p.labels, dev)
    alpha, lam, st = pl.solve(y, 2.0)
    assert st["status"] == 0
    return p, pl, y, alpha, lam


def test_decision_function_at_new_points_matches_oracle(dev, trained):
    import paper_2312_00538_amd as lib
    p, pl, y, alpha, lam = trained
    q = workloads.gaussian_mixture(seed=7, N=1200, d=9, R=0)
    Xn = q.X[:400] * 1.3          # new points, partly outside the training range
    f = lib.decision_function(to_dev(p.X, dev), to_dev(Xn, dev), p.windows, p.sigma, y, alpha, lam).cpu().numpy()
    a = alpha.cpu().numpy()
    kpart = oracle.anova_cross(Xn, p.X, p.windows, p.sigma, p.labels * a)
    rel = np.linalg.norm(f + lam - kpart) / np.linalg.norm(kpart)
    print("rel err of K(Xnew, X) y alpha:", rel)
    assert rel <= 1e-6
    ref = kpart - lam
    sure = np.abs(ref) > 1e-3
    assert np.array_equal(np.sign(f[sure]), np.sign(ref[sure]))


def test_decision_function_at_the_training_points(dev, trained):
    # targets = sources: f = K Y alpha - lambda, as the training plan computes it
    import paper_2312_00538_amd as lib
    p, pl, y, alpha, lam = trained
    f = lib.decision_function(to_dev(p.X, dev), to_dev(p.X, dev), p.windows, p.sigma, y, alpha, lam).cpu().numpy()
    kya = pl.matvec(y * alpha).cpu().numpy()
    rel = np.linalg.norm(f + lam - kya) / np.linalg.norm(kya)
    print("rel diff to the training plan:", rel)
    assert rel <= 1e-7


def test_decision_function_rejects_bad_shapes(dev, trained):
    import paper_2312_00538_amd as lib
    p, pl, y, alpha, lam = trained
    with pytest.raises(ValueError):
        lib.decision_function(to_dev(p.X, dev), to_dev(p.X[:, :5].copy(), dev), p.windows, p.sigma, y, alpha, lam)
