"""GPU parity of the variants, through the C ABI, against the FP64 oracle.

* Generalized ADMM baseline (Step 4 replaced by the rho-relaxation, Sec. 4.1):
  fixed trajectories equal the oracle's after k updates; converged solves
  take the same iterations and reach the same objective.
* Absolute KKT stopping (||R(w_bar)|| of Prop. complexity): the reported
  residual equals the oracle's, and the stop happens at the same iteration.
"""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu


def close(a, b, tol, floor):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max()) <= tol * max(float(np.abs(b).max()), floor)

pytestmark = pytest.mark.gpu


def hist(rng, m, n, zeros=0.0):
    h = rng.uniform(0.05, 1.0, size=(m, n))
    if zeros:
        h[rng.uniform(size=(m, n)) < zeros] = 0
        if h.sum() == 0:
            h[0, 0] = 1
    return h / h.sum()


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (7, 5), (32, 32), (17, 40)])
@pytest.mark.parametrize("k", [1, 10, 100])
@pytest.mark.parametrize("rho", [1.7, 1.0])
def test_admm_fixed_trajectory(oracle, m, n, k, rho):
    need_gpu()
    from paper_2408_00598_amd import hot
    rng = np.random.default_rng(11 * m + n + k)
    mu1, mu2 = hist(rng, m, n, 0.1), hist(rng, m, n, 0.1)
    c = ctx()
    res, sol = c.solve(dev(mu1), dev(mu2), keep=True, max_iter=k, relax=rho,
                       flags=hot.HOT_FLAG_FIXED_ITERS | hot.HOT_FLAG_ADMM)
    xb, yb, zb, s = (t.cpu().numpy() for t in sol.export())
    oxb, oyb, ozb, os_, ores = oracle.hot(mu1, mu2, fixed_iters=k, restart=False,
                                          admm_rho=rho)
    assert res["iters"] == k
    # y and z live on the cost scale (integer costs, 0 on a 1 x 1 grid where
    # y is rounding noise), x and s on the mass scale: floors of 1 and 1e-3
    assert close(s, os_, 1e-10, 1e-3)
    assert close(yb, oyb, 1e-10, 1.0)
    assert close(xb, oxb, 1e-9, 1e-3)
    assert close(zb, ozb, 1e-9, 1.0)
    assert abs(res["kkt_abs"] - ores["kkt_abs"]) <= 1e-9 * ores["kkt_abs"] + 1e-14


@pytest.mark.parametrize("m,n,tol", [(8, 8, 1e-6), (32, 32, 1e-4), (12, 20, 1e-6)])
def test_admm_converged(oracle, m, n, tol):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(0, 3 * m + n))
    mu1, mu2 = workloads.gaussian_blobs(m, n, 3, rng), workloads.gaussian_blobs(m, n, 3, rng)
    c = ctx()
    res, _ = c.solve(dev(mu1), dev(mu2), tol=tol, max_iter=400000,
                     flags=hot.HOT_FLAG_ADMM)  # relax <= 0 selects 1.7
    _, _, _, _, ores = oracle.hot(mu1, mu2, tol=tol, max_iter=400000, admm_rho=1.7)
    assert res["status"] == 0 and ores["converged"] == 1
    assert res["restarts"] == 0
    assert res["iters"] == ores["iters"]
    assert abs(res["primal_obj"] - ores["primal_obj"]) <= 1e-6 * abs(ores["primal_obj"])
    assert res["kkt"] <= tol


@pytest.mark.parametrize("flags_name,rho,m,n", [("HOT_FLAG_RESTART", 0.0, 8, 8),
                                                ("HOT_FLAG_RESTART", 0.0, 16, 24),
                                                ("HOT_FLAG_ADMM", 1.7, 8, 8)])
def test_absolute_kkt_stop(oracle, flags_name, rho, m, n):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(0, 5 * m + n))
    mu1, mu2 = workloads.gaussian_blobs(m, n, 3, rng), workloads.gaussian_blobs(m, n, 3, rng)
    tol = 1e-6
    c = ctx()
    flags = getattr(hot, flags_name) | hot.HOT_FLAG_ABS_KKT
    res, _ = c.solve(dev(mu1), dev(mu2), tol=tol, max_iter=400000, flags=flags, relax=rho)
    _, _, _, _, ores = oracle.hot(mu1, mu2, tol=tol, max_iter=400000, abs_kkt=True,
                                  admm_rho=rho)
    assert res["status"] == 0 and ores["converged"] == 1
    assert res["iters"] == ores["iters"]
    assert res["restarts"] == ores["restarts"]
    assert res["kkt_abs"] <= tol
    assert abs(res["kkt_abs"] - ores["kkt_abs"]) <= 1e-6 * ores["kkt_abs"]
    assert abs(res["primal_obj"] - ores["primal_obj"]) <= 1e-6 * abs(ores["primal_obj"])


def test_admm_relax_out_of_range_rejected():
    need_gpu()
    from paper_2408_00598_amd import hot
    c = ctx()
    mu = np.full((4, 4), 1 / 16)
    for bad in (2.0, 3.5, float("nan")):
        with pytest.raises(hot.HotError):
            c.solve(dev(mu), dev(mu), flags=hot.HOT_FLAG_ADMM, relax=bad)
