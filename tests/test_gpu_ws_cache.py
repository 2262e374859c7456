"""The context's workspace cache: a solve or batch that takes over the
workspace of an earlier call of the same shapes (set up afresh, graph kept)
gives bit-for-bit the result of a context that never solved before, whatever
the earlier call's flags (sigma re-balancing, non-uniform bins) were."""
import numpy as np
import pytest

from gpu_helpers import dev, need_gpu

pytestmark = pytest.mark.gpu

KEYS = ("primal_obj", "dual_obj", "kkt", "kkt_abs", "feaserr", "iters", "restarts", "status")


def pair(m, n, seed):
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(workloads.seed_for(6, seed))
    return dev(workloads.gaussian_blobs(m, n, 3, rng)), dev(workloads.gaussian_blobs(m, n, 2, rng))


def test_solves_through_the_cache_equal_fresh():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    R, SU = hot.HOT_FLAG_RESTART, hot.HOT_FLAG_SIGMA_UPDATE
    rng = np.random.default_rng(3)
    cu, cv = dev(workloads.grid_lines(40, rng)), dev(workloads.grid_lines(48, rng))
    calls = [  # one shape, different flags, repeated
        (pair(40, 48, 1), dict(tol=1e-6, flags=R)),
        (pair(40, 48, 2), dict(tol=1e-6, flags=R | SU)),
        (pair(40, 48, 3), dict(tol=1e-6, flags=R, coord_row=cu, coord_col=cv)),
        (pair(40, 48, 1), dict(tol=1e-6, flags=R)),
        (pair(40, 48, 4), dict(tol=1e-4, flags=R, prec=hot.HOT_FP32_STREAM)),
        (pair(40, 48, 2), dict(tol=1e-6, flags=R | SU)),
    ]
    cached = hot.Context(0)
    for q, ((a, b), kw) in enumerate(calls):
        print(f"cache call {q}: {kw.get('flags')} prec={kw.get('prec', 0)}", flush=True)
        got, _ = cached.solve(a, b, max_iter=200000, **kw)
        fresh_ctx = hot.Context(0)
        want, _ = fresh_ctx.solve(a, b, max_iter=200000, **kw)
        fresh_ctx.close()
        assert want["status"] == hot.HOT_OK
        for k in KEYS:
            assert got[k] == want[k], (q, k, got[k], want[k])


def test_batches_through_the_cache_equal_fresh():
    need_gpu()
    from paper_2408_00598_amd import hot
    shapes = [(32, 32), (48, 40), (64, 64), (24, 56)]
    cached = hot.Context(0)
    for rep in range(3):
        pairs = [pair(m, n, 10 * rep + q) for q, (m, n) in enumerate(shapes)]
        print(f"cache batch {rep}", flush=True)
        got = cached.batch_solve(pairs, tol=1e-4, max_iter=100000, prec=hot.HOT_FP32_STREAM)
        fresh_ctx = hot.Context(0)
        want = fresh_ctx.batch_solve(pairs, tol=1e-4, max_iter=100000, prec=hot.HOT_FP32_STREAM)
        fresh_ctx.close()
        for q in range(len(shapes)):
            assert want[q]["status"] == hot.HOT_OK
            for k in KEYS:
                assert got[q][k] == want[q][k], (rep, q, k)
