"""GPU tests of the autotuner (bandwidth, cutoff, precision and work-item size
chosen per data set): the chosen options meet the target error against the
FP64 oracle, the choice is the fastest admissible candidate, and candidates
above the target are not timed."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.mark.parametrize("target,rhs", [(1e-4, 1), (1e-4, 16), (1e-7, 1)])
def test_autotune_choice_meets_the_target(dev, target, rhs):
    import paper_2312_00538_amd as lib
    p = workloads.gaussian_mixture(seed=9, N=20_000, d=9, R=rhs, sigma=0.6)
    X = to_dev(p.X, dev)
    best, cands, chosen = lib.autotune(X, p.windows, p.sigma, target_rel_err=target, rhs=rhs)
    for c in cands:
        print(c)
    print("chosen", chosen, cands[chosen])
    timed = [c for c in cands if c["ms"] >= 0]
    assert all(0 <= c["rel_err"] <= target for c in timed)
    assert all(c["ms"] < 0 for c in cands if c["rel_err"] > target)
    assert cands[chosen]["ms"] == min(c["ms"] for c in timed)
    # the chosen options against the oracle on sampled rows
    pl = lib.Plan(X, p.windows, p.sigma, opts=best)
    y = pl.matvec(to_dev(p.v[:, :rhs], dev)).cpu().numpy().reshape(p.X.shape[0], rhs)[:, 0]
    rows = np.random.default_rng(1).choice(p.X.shape[0], 256, replace=False)
    ref = oracle.anova_matvec(p.X, p.windows, p.sigma, p.v[:, 0], rows=rows).reshape(-1)
    err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
    print("oracle rel err of the choice", err)
    assert err <= 2 * target + 2e-8   # the reference plan's own error is ~1e-8
