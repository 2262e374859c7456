"""hot_solve_noalloc (the entry point for callers that cannot allocate)
against hot_solve, through the C ABI: the same kernels over a workspace carved
from the library's static device array, so the result and the final iterate
must be bit-identical to hot_solve's.  Two calls in a row, the second on a
smaller problem (the array keeps the first call's contents), and a problem
too large for the array is refused with a clear error.
"""
import numpy as np
import pytest

from gpu_helpers import dev, need_gpu

pytestmark = pytest.mark.gpu

KEYS = ("primal_obj", "dual_obj", "kkt", "res_primal", "res_dual", "res_comp", "kkt_abs",
        "feaserr", "sigma", "iters", "restarts", "status")


def same_as_solve(c, mu1, mu2, **kw):
    import torch
    d1, d2 = dev(mu1), dev(mu2)
    ra, xa, ya = c.solve_noalloc(d1, d2, **kw)
    rb, sol = c.solve(d1, d2, keep=True, **kw)
    xb, yb, _, _ = sol.export()
    sol.free()
    print("noalloc", mu1.shape, kw, ra["iters"], ra["status"], flush=True)
    for key in KEYS:
        assert ra[key] == rb[key], (key, ra[key], rb[key])
    assert torch.equal(xa, xb) and torch.equal(ya, yb)
    return ra


def test_noalloc_equals_solve_two_calls():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = hot.Context(0)
    rng = np.random.default_rng(workloads.seed_for(5, 1))
    # first call: 96 x 96 FP32 streams, converged with restarts
    a, b = workloads.gaussian_blobs(96, 96, 4, rng), workloads.gaussian_blobs(96, 96, 4, rng)
    r1 = same_as_solve(c, a, b, tol=1e-4, max_iter=50000, prec=hot.HOT_FP32_STREAM)
    assert r1["status"] == 0 and r1["restarts"] >= 1
    # second call, smaller and in FP64, on the array the first call left behind
    a, b = workloads.gaussian_blobs(17, 23, 3, rng), workloads.gaussian_blobs(17, 23, 3, rng)
    r2 = same_as_solve(c, a, b, tol=1e-6, max_iter=200000)
    assert r2["status"] == 0
    # fixed iterations and sigma re-balancing go through the same path
    same_as_solve(c, a, b, max_iter=37, flags=hot.HOT_FLAG_FIXED_ITERS)
    same_as_solve(c, a, b, tol=1e-6, max_iter=200000,
                  flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE)


def test_noalloc_rejects_oversize():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = hot.Context(0)
    cap = int(hot.lib().hot_noalloc_capacity())
    assert cap == 64 << 20
    assert hot.footprint_bytes(256, 256, hot.HOT_FP32_STREAM) > cap
    rng = np.random.default_rng(3)
    a, b = workloads.gaussian_blobs(256, 256, 3, rng), workloads.gaussian_blobs(256, 256, 3, rng)
    with pytest.raises(hot.HotError) as e:
        c.solve_noalloc(dev(a), dev(b), tol=1e-4, prec=hot.HOT_FP32_STREAM)
    assert e.value.status == hot.HOT_E_INVALID and "no-alloc" in c.last_error()
    # and the context still works afterwards
    a, b = workloads.pair_small(2)
    same_as_solve(c, a, b, tol=1e-6)
