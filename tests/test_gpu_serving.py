"""GPU tests of the request server (continuous batching of IPM solves of
different sizes): results equal the one-at-a-time solve and do not depend on
the mix, admission follows the memory budget, matvecs of resident solves share
launches, and bad requests are reported to their caller."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _problem(seed, N, d, sigma=1.0, C=1.0):
    p = workloads.gaussian_mixture(seed=seed, N=N, d=d, sigma=sigma, C=C, R=0)
    return p


def _direct(p, dev):
    import paper_2312_00538_amd as lib
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    alpha, lam, st = pl.solve(to_dev(p.labels, dev), p.C, allow_not_converged=True)
    return alpha.cpu().numpy(), lam, st


MIX = [(11, 900, 7, 0.8, 1.0), (12, 2500, 12, 1.2, 5.0), (13, 1600, 6, 0.6, 0.5), (14, 3100, 9, 1.0, 2.0)]


def test_server_result_equals_direct_solve(dev):
    import paper_2312_00538_amd as lib
    p = _problem(*MIX[0])
    a_ref, lam_ref, st_ref = _direct(p, dev)
    srv = lib.Server(max_active=4)
    t = srv.submit(p.X, p.labels, p.windows, p.sigma, p.C)
    a, res = srv.wait(t)
    srv.close()
    print("direct", st_ref["ip_iters"], st_ref["rel_gap"], "served", res["stats"]["ip_iters"], res["latency_ms"])
    assert res["status"] == 0
    assert np.array_equal(a, a_ref)
    assert res["lambda"] == lam_ref
    assert res["stats"]["ip_iters"] == st_ref["ip_iters"]


@pytest.mark.parametrize("share", [True, False])
def test_same_alone_and_in_the_mix(dev, share):
    import paper_2312_00538_amd as lib
    probs = [_problem(*m) for m in MIX]
    alone = []
    srv = lib.Server(max_active=1, share_launches=share)
    for p in probs:
        alone.append(srv.wait(srv.submit(p.X, p.labels, p.windows, p.sigma, p.C)))
    srv.close()
    srv = lib.Server(max_active=4, share_launches=share)
    tickets = [srv.submit(p.X, p.labels, p.windows, p.sigma, p.C) for p in probs]
    mixed = [srv.wait(t) for t in tickets]
    launches, matvecs = srv.counters()
    srv.close()
    for (a1, r1), (a2, r2) in zip(alone, mixed):
        assert r1["status"] == 0 and r2["status"] == 0
        assert np.array_equal(a1, a2)
        assert r1["lambda"] == r2["lambda"]
        assert r1["stats"]["ip_iters"] == r2["stats"]["ip_iters"]
    print(f"share={share}: {matvecs} matvecs in {launches} shared launches")
    if share:
        assert matvecs > launches   # some matvecs of different solves went out together


def test_admission_follows_the_memory_budget(dev):
    import paper_2312_00538_amd as lib
    probs = [_problem(*m) for m in MIX[:2]]
    fps = [lib.request_footprint(p.X.shape[0], p.X.shape[1], p.windows.shape[0]) for p in probs]
    # room for either request alone but not for both
    srv = lib.Server(max_active=8, hbm_budget=max(fps) + min(fps) // 2)
    t = [srv.submit(p.X, p.labels, p.windows, p.sigma, p.C) for p in probs]
    r = [srv.wait(x)[1] for x in t]
    srv.close()
    print([(x["queue_ms"], x["run_ms"]) for x in r])
    assert r[0]["footprint"] == fps[0] and r[1]["footprint"] == fps[1]
    assert r[1]["queue_ms"] >= 0.9 * r[0]["run_ms"]       # admitted only after the first finished
    # with room for both, the second starts at once
    srv = lib.Server(max_active=8, hbm_budget=2 * sum(fps))
    t = [srv.submit(p.X, p.labels, p.windows, p.sigma, p.C) for p in probs]
    r = [srv.wait(x)[1] for x in t]
    srv.close()
    assert r[1]["queue_ms"] < 0.5 * r[0]["run_ms"]


def test_bad_request_is_reported_at_wait(dev):
    import paper_2312_00538_amd as lib
    p = _problem(*MIX[0])
    srv = lib.Server(max_active=2)
    bad = srv.submit(p.X, np.ones_like(p.labels), p.windows, p.sigma, p.C)   # one class only
    good = srv.submit(p.X, p.labels, p.windows, p.sigma, p.C)
    with pytest.raises(lib.AnovaError) as e:
        srv.wait(bad)
    assert e.value.status == lib.INVALID_ARG
    a, res = srv.wait(good)
    assert res["status"] == 0
    with pytest.raises(lib.AnovaError):
        srv.submit(p.X, p.labels, p.windows, p.sigma, -1.0)
    srv.close()


def test_served_results_meet_the_exact_qp_bar(dev):
    # every request of the mix, served concurrently with shared launches, is
    # evaluated in the exact QP of Algorithm 1 (eq. "kernelsvm") with a dense K:
    # relative duality gap G_exact <= 1e-6, and the dual objective within 1e-6
    # (relative) of the dense-KKT oracle's optimum
    import paper_2312_00538_amd as lib
    probs = [_problem(*m) for m in MIX]
    srv = lib.Server(max_active=4, share_launches=True)
    tickets = [srv.submit(p.X, p.labels, p.windows, p.sigma, p.C) for p in probs]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for p, (a, res) in zip(probs, served):
        assert res["status"] == 0
        K = oracle.anova_dense(p.X, p.windows, p.sigma)
        ref = oracle.ipm_dense(K, p.labels, p.C)
        assert ref["converged"]
        D, Pr, G = oracle.objectives_from_kya(K @ (p.labels * a), p.labels, a, res["lambda"], p.C)
        rel_d = abs(D - ref["D"]) / abs(ref["D"])
        print(f"N={p.X.shape[0]} d={p.X.shape[1]} C={p.C}: G_exact {G:.2e}, dual {D:.10g} vs oracle "
              f"{ref['D']:.10g} (rel {rel_d:.2e}), |y^T a| {abs(p.labels @ a):.1e}")
        assert G <= 1e-6
        assert rel_d <= 1e-6
