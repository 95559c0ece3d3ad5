"""GPU parity of the IPM with GMRES and the block-triangular preconditioner
P = [[A_hat, 0], [-y^T, -1]] of Section 5.

The first IPM steps from Algorithm 1's starting point, with the Krylov
tolerance at its floor (1e-10), follow the dense-KKT oracle's steps; the
remaining difference is the fast summation's error in K amplified by the
Newton matrix (condition number about 2.5e3 on this problem), about 1e-7 C
after three steps, so alpha is compared to 1e-6 C there, and GMRES to MINRES,
on the same operator (a difference of a few 1e-9 C), to 1e-7 C.
Full solves meet the IPM bar of the MINRES tests: the GPU's own relative gap
<= 1e-6, G_exact <= 1e-6 in the exact QP and the dual objective within 1e-6 of
the oracle's."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device, to_dev
from test_gpu_solver import _check_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _first_steps(lib, p, dev, krylov, precond, steps, **kw):
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    alpha, lam, st = pl.solve(to_dev(p.labels, dev), 1.0, krylov=krylov, precond=precond, max_ip=steps,
                              tol_kry=1e-10, allow_not_converged=True, **kw)
    return alpha.cpu().numpy(), lam, st


@pytest.mark.parametrize("precond", ["none", "diag", "pchol"])
def test_first_newton_steps_follow_the_dense_oracle(dev, precond):
    import paper_2312_00538_amd as lib
    pc = {"none": lib.PRECOND_NONE, "diag": lib.PRECOND_DIAG, "pchol": lib.PRECOND_PCHOL}[precond]
    # without a preconditioner, max_kry = 10 restarts GMRES every 10 steps
    kw = dict(max_kry=10) if precond == "none" else dict(rank=100)
    p = workloads.small_plain(seed=0, N=300)
    K = oracle.anova_dense(p.X, p.windows, p.sigma)
    for steps in (1, 3):
        ref = oracle.ipm_dense(K, p.labels, 1.0, max_ip=steps)
        ag, lg, sg = _first_steps(lib, p, dev, lib.KRYLOV_GMRES, pc, steps, **kw)
        am, lm, sm = _first_steps(lib, p, dev, lib.KRYLOV_MINRES, pc, steps, **kw)
        print(precond, steps, "gmres", sg["kry_iters_total"], sg["kry_iters_max"], "minres", sm["kry_iters_total"],
              "d_oracle", np.max(np.abs(ag - ref["alpha"])), abs(lg - ref["lam"]), "d_minres", np.max(np.abs(ag - am)))
        assert sg["ip_iters"] == steps and np.isfinite(ag).all()
        assert np.max(np.abs(ag - ref["alpha"])) <= 1e-6
        assert abs(lg - ref["lam"]) <= 1e-6 * max(1.0, abs(ref["lam"]))
        assert np.max(np.abs(ag - am)) <= 1e-7
        if precond == "none" and steps == 3:
            assert sg["kry_iters_max"] > 10     # at least one restart


@pytest.mark.parametrize("precond", ["diag", "pchol"])
def test_ipm_gmres_small_plain_parity(dev, precond):
    import paper_2312_00538_amd as lib
    p = workloads.small_plain(seed=0, N=2000, d=9)
    pc = {"diag": lib.PRECOND_DIAG, "pchol": lib.PRECOND_PCHOL}[precond]
    a, lam, st = _check_solve(p, 1.0, dev, precond=pc, krylov=lib.KRYLOV_GMRES)
    print("gmres krylov", st["kry_iters_total"], st["kry_iters_max"])


@pytest.mark.parametrize("precond", ["pchol", "nystrom"])
def test_ipm_gmres_mixture_parity(dev, precond):
    import paper_2312_00538_amd as lib
    p = workloads.gaussian_mixture(seed=1, N=600, d=20, noise=0.1, sigma=0.8, C=10.0)
    pc = {"pchol": lib.PRECOND_PCHOL, "nystrom": lib.PRECOND_NYSTROM}[precond]
    a, lam, st = _check_solve(p, 10.0, dev, rank=100, precond=pc, seed=3, krylov=lib.KRYLOV_GMRES)
    print("gmres krylov", st["kry_iters_total"], st["kry_iters_max"])
    assert st["kry_iters_max"] <= 20


def test_ipm_gmres_deterministic(dev):
    import paper_2312_00538_amd as lib
    p = workloads.small_plain(seed=5, N=700)
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    y = to_dev(p.labels, dev)
    a1, l1, s1 = pl.solve(y, 1.0, rank=100, krylov=lib.KRYLOV_GMRES)
    a2, l2, s2 = pl.solve(y, 1.0, rank=100, krylov=lib.KRYLOV_GMRES)
    assert np.array_equal(a1.cpu().numpy(), a2.cpu().numpy()) and l1 == l2
    assert s1["kry_iters_total"] == s2["kry_iters_total"]


def test_server_gmres_equals_direct_solve(dev):
    # matvecs through the server's shared launches: the same iterates bit for bit
    import paper_2312_00538_amd as lib
    p = workloads.gaussian_mixture(seed=11, N=900, d=7, sigma=0.8, C=1.0, R=0)
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    a_ref, lam_ref, st_ref = pl.solve(to_dev(p.labels, dev), p.C, krylov=lib.KRYLOV_GMRES)
    srv = lib.Server(max_active=2)
    t = srv.submit(p.X, p.labels, p.windows, p.sigma, p.C, krylov=lib.KRYLOV_GMRES)
    u = srv.submit(p.X, p.labels, p.windows, p.sigma, p.C)      # a MINRES solve alongside
    a, res = srv.wait(t)
    a2, res2 = srv.wait(u)
    srv.close()
    print("direct", st_ref["kry_iters_total"], "served", res["stats"]["kry_iters_total"],
          "minres", res2["stats"]["kry_iters_total"])
    assert res["status"] == 0 and res2["status"] == 0
    assert np.array_equal(a, a_ref.cpu().numpy())
    assert res["lambda"] == lam_ref


def test_unknown_krylov_method_is_rejected(dev):
    import paper_2312_00538_amd as lib
    p = workloads.small_plain(seed=0, N=300)
    pl = lib.Plan(to_dev(p.X, dev), p.windows, p.sigma)
    with pytest.raises(lib.AnovaError) as e:
        pl.solve(to_dev(p.labels, dev), 1.0, krylov=2)
    assert e.value.status == lib.INVALID_ARG
