"""Optional sigma re-balancing at restarts (HOT_FLAG_SIGMA_UPDATE) on the GPU
path against the oracle: sigma <- ||x_bar - X|| / ||A^T (y_bar - Y)|| over
each epoch, (X, Y) the w_bar of the previous restart.  The check pass adds
||x_bar - X||^2 (one more stream), the reduce adds ||A^T dy||^2 per slab in
closed form, and the restart pass writes x_bar / sigma_new + z_bar."""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def case(m, n, kind="b"):
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(workloads.seed_for(5, m + n))
    if kind == "b":
        return workloads.gaussian_blobs(m, n, 3, rng), workloads.gaussian_blobs(m, n, 3, rng)
    return workloads.white_noise(m, n, rng), workloads.white_noise(m, n, rng)


@pytest.mark.parametrize("m,n,tol,kind", [(16, 16, 1e-6, "b"), (24, 20, 1e-6, "b"),
                                          (12, 28, 1e-6, "n"), (32, 32, 1e-4, "b"),
                                          (16, 16, 1e-9, "b")])
def test_sigma_update_matches_oracle_fp64(oracle, m, n, tol, kind):
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2 = case(m, n, kind)
    c = ctx()
    res, _ = c.solve(dev(mu1), dev(mu2), tol=tol, max_iter=400000,
                     flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE)
    o = oracle.hot(mu1, mu2, tol=tol, max_iter=400000, sigma_update=True)[4]
    assert res["status"] == 0 and o["converged"] == 1 and o["restarts"] >= 2
    assert res["iters"] == o["iters"] and res["restarts"] == o["restarts"]
    # sigma is a ratio of norms of differences of nearly converged iterates
    # (||x_bar - X|| ~ 1e-7 ||x_bar|| at tol 1e-9), so rounding in the two
    # summation orders reaches it at ~1e-16 ||x_bar|| / ||x_bar - X||
    assert abs(res["sigma"] - o["sigma"]) <= 1e-7 * o["sigma"]
    assert abs(res["primal_obj"] - o["primal_obj"]) <= 1e-6 * abs(o["primal_obj"])


def test_sigma_update_fp32_streams(oracle):
    """FP32 streams keep X in FP32, so sigma (and the iterate path) differs
    from FP64 by rounding; the result must be as accurate as the oracle's
    own at the same tolerance: |obj32 - opt| <= 2 |obj_or - opt| + 1e-4 opt."""
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2 = case(24, 20)
    c = ctx()
    res, _ = c.solve(dev(mu1), dev(mu2), tol=1e-6, max_iter=400000, prec=hot.HOT_FP32_STREAM,
                     flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE)
    o = oracle.hot(mu1, mu2, tol=1e-6, max_iter=400000, sigma_update=True)[4]["primal_obj"]
    opt = oracle.hot(mu1, mu2, tol=1e-9, max_iter=400000)[4]["primal_obj"]
    assert res["status"] == 0 and res["restarts"] >= 2
    assert abs(res["primal_obj"] - opt) <= 2 * abs(o - opt) + 1e-4 * abs(opt)


def test_sigma_update_batch_equals_solo():
    need_gpu()
    from paper_2408_00598_amd import hot
    c = ctx()
    su = hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE
    cases = [case(12, 12), case(16, 8), case(9, 14, "n"), case(10, 10)]
    pairs = [(dev(a), dev(b), {"flags": su if i % 2 == 0 else hot.HOT_FLAG_RESTART})
             for i, (a, b) in enumerate(cases)]
    batch = c.batch_solve(pairs, tol=1e-6, max_iter=200000)
    for (a, b, extra), rb in zip(pairs, batch):
        ra, _ = c.solve(a, b, tol=1e-6, max_iter=200000, **extra)
        assert ra["status"] == 0 and rb["status"] == 0
        assert ra["iters"] == rb["iters"] and ra["restarts"] == rb["restarts"]
        assert abs(ra["sigma"] - rb["sigma"]) <= 1e-12 * ra["sigma"]
        assert abs(ra["primal_obj"] - rb["primal_obj"]) <= 1e-12 * abs(ra["primal_obj"])


def test_sigma_update_ignored_without_restarts():
    """The flag acts at restarts only: with fixed iterations (or the ADMM
    baseline) the result is bit-identical to the run without it."""
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2 = case(12, 10)
    c = ctx()
    for base in (hot.HOT_FLAG_FIXED_ITERS, hot.HOT_FLAG_ADMM):
        kw = dict(max_iter=60, tol=1e-6)
        a, _ = c.solve(dev(mu1), dev(mu2), flags=base, raise_on_error=False, **kw)
        b, _ = c.solve(dev(mu1), dev(mu2), flags=base | hot.HOT_FLAG_SIGMA_UPDATE,
                       raise_on_error=False, **kw)
        for key in ("primal_obj", "dual_obj", "kkt", "iters", "sigma"):
            assert a[key] == b[key], (base, key)
