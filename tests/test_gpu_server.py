"""Continuous-batching service: problems submitted while others are resident
are admitted as slots and HBM budget free up, run concurrently, and each
result is identical to the same problem solved alone."""
import time

import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def test_server_results_equal_alone_and_overlap():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = ctx()
    srv = hot.Server(c, hbm_budget_bytes=0, max_slots=3)
    reqs = []
    rng = np.random.default_rng(11)
    for t in range(9):
        n = (16, 24, 32)[t % 3]
        a = workloads.gaussian_blobs(n, n, 2, rng)
        b = workloads.gaussian_blobs(n, n, 3, rng)
        tol = 1e-4 if t % 2 else 1e-6
        prec = hot.HOT_FP32_STREAM if t % 4 == 1 else hot.HOT_FP64
        reqs.append((t, dev(a), dev(b), tol, prec))
    for q, (t, a, b, tol, prec) in enumerate(reqs):
        srv.submit(a, b, t, tol=tol, prec=prec, max_iter=200000)
        if q in (2, 5):
            time.sleep(0.01)  # later arrivals join a running mix
    assert srv.drain(300.0) == hot.HOT_OK
    got = {r["tag"]: r for r in srv.poll(64)}
    st = srv.stats()
    srv.close()
    assert len(got) == len(reqs)
    assert st["max_resident"] >= 2 and st["max_resident"] <= 3
    assert st["p99"] >= st["p50"] > 0
    for t, a, b, tol, prec in reqs:
        alone, _ = c.solve(a, b, tol=tol, prec=prec, max_iter=200000)
        r = got[t]
        for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
            assert r[key] == alone[key], (t, key, r[key], alone[key])


def test_server_admission_respects_budget():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = ctx()
    fp = hot.footprint_bytes(32, 32, hot.HOT_FP64)
    srv = hot.Server(c, hbm_budget_bytes=int(2.5 * fp), max_slots=8)
    pairs = [workloads.pair_small(p) for p in range(5)]
    keep = [(dev(a), dev(b)) for a, b in pairs]
    for t, (a, b) in enumerate(keep):
        srv.submit(a, b, t, tol=1e-5, max_iter=200000)
    assert srv.drain(300.0) == hot.HOT_OK
    res = srv.poll(16)
    st = srv.stats()
    srv.close()
    assert len(res) == 5 and all(r["status"] == 0 for r in res)
    assert st["max_resident"] == 2
    # mixed shapes and precisions, admitted by the context's footprints:
    # any three of them exceed the budget, any two fit
    shapes = [(40, 40, hot.HOT_FP64), (36, 44, hot.HOT_FP64), (44, 36, hot.HOT_FP64),
              (52, 50, hot.HOT_FP32_STREAM)]
    fps = sorted(c.footprint_bytes(m, n, p) for m, n, p in shapes)
    assert all(f > 0 for f in fps)
    budget = fps[-1] + fps[-2]
    assert fps[0] + fps[1] + fps[2] > budget
    srv = hot.Server(c, hbm_budget_bytes=budget, max_slots=8)
    rng = np.random.default_rng(5)
    keep2 = []
    for t, (m, n, p) in enumerate(shapes):
        a, b = dev(workloads.gaussian_blobs(m, n, 2, rng)), dev(workloads.gaussian_blobs(m, n, 2, rng))
        keep2.append((a, b))
        srv.submit(a, b, t, tol=1e-5, prec=p, max_iter=200000)
    assert srv.drain(300.0) == hot.HOT_OK
    res = srv.poll(16)
    st = srv.stats()
    srv.close()
    assert len(res) == 4 and all(r["status"] == 0 for r in res)
    assert st["max_resident"] <= 2
    # a problem larger than the whole budget is refused at submission
    srv = hot.Server(c, hbm_budget_bytes=fp // 2, max_slots=2)
    with pytest.raises(hot.HotError):
        srv.submit(*keep[0], 99, tol=1e-5)
    srv.close()


def test_server_shared_launches_equal_alone():
    """HOT_SERVER_SHARED: problems of one class iterate in the same launches
    (slots of one group, joined at quantum boundaries while others run), and
    each result is still bit-identical to its solo hot_solve result."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = ctx()
    srv = hot.Server(c, hbm_budget_bytes=0, max_slots=5, shared=True)
    rng = np.random.default_rng(21)
    reqs = []
    shapes = [(32, 32), (24, 24), (17, 30), (32, 32), (40, 40), (48, 33), (64, 64), (60, 50),
              (32, 9), (20, 20), (64, 64), (45, 48)]
    for t, (m, n) in enumerate(shapes):
        a = workloads.gaussian_blobs(m, n, 2, rng)
        b = workloads.gaussian_blobs(m, n, 3, rng)
        tol = 1e-4 if t % 3 else 1e-6
        prec = hot.HOT_FP32_STREAM if t % 2 else hot.HOT_FP64
        flags = hot.HOT_FLAG_RESTART | (hot.HOT_FLAG_SIGMA_UPDATE if t % 5 == 4 else 0)
        reqs.append((t, dev(a), dev(b), tol, prec, flags))
    for q, (t, a, b, tol, prec, flags) in enumerate(reqs):
        srv.submit(a, b, t, tol=tol, prec=prec, max_iter=200000, flags=flags)
        if q in (3, 7):
            time.sleep(0.02)  # later arrivals join groups that are running
    assert srv.drain(300.0) == hot.HOT_OK
    got = {r["tag"]: r for r in srv.poll(64)}
    st = srv.stats()
    srv.close()
    assert len(got) == len(reqs)
    assert st["max_shared"] >= 2 and st["max_resident"] <= 5
    for t, a, b, tol, prec, flags in reqs:
        alone, _ = c.solve(a, b, tol=tol, prec=prec, max_iter=200000, flags=flags)
        r = got[t]
        assert r["status"] == hot.HOT_OK, (t, r["status"])
        for key in ("primal_obj", "dual_obj", "kkt", "kkt_abs", "feaserr", "iters", "restarts",
                    "status"):
            assert r[key] == alone[key], (t, key, r[key], alone[key])


def test_server_shared_slots_reused():
    """More same-class requests than slots: slots are freed and reused at
    quantum boundaries; every result equals its solo result."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = ctx()
    srv = hot.Server(c, max_slots=2, shared=True)
    pairs = []
    for t in range(7):
        a, b = workloads.serving_pair(64, workloads.seed_for(9, t))
        pairs.append((dev(a), dev(b)))
        srv.submit(*pairs[-1], t, tol=1e-4, prec=hot.HOT_FP32_STREAM, max_iter=100000)
    assert srv.drain(300.0) == hot.HOT_OK
    got = {r["tag"]: r for r in srv.poll(64)}
    st = srv.stats()
    srv.close()
    assert st["max_shared"] == 2 and st["max_resident"] <= 2
    for t, (a, b) in enumerate(pairs):
        alone, _ = c.solve(a, b, tol=1e-4, prec=hot.HOT_FP32_STREAM, max_iter=100000)
        for key in ("primal_obj", "kkt", "iters", "feaserr", "status"):
            assert got[t][key] == alone[key], (t, key)


def test_server_shared_variants_equal_alone():
    """Shared launches with the method's variants in one group: non-uniform
    bins beside uniform ones, the ADMM baseline, absolute-KKT stopping and
    fixed iterations; each result equals its solo hot_solve result."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = ctx()
    rng = np.random.default_rng(33)
    R = hot.HOT_FLAG_RESTART
    specs = [  # (m, n, prec, tol, flags, max_iter, non-uniform)
        (40, 40, hot.HOT_FP64, 1e-6, R, 200000, True),
        (44, 40, hot.HOT_FP64, 1e-6, R, 200000, False),
        (48, 36, hot.HOT_FP64, 1e-5, hot.HOT_FLAG_ADMM, 200000, False),
        (40, 48, hot.HOT_FP64, 1e-3, R | hot.HOT_FLAG_ABS_KKT, 200000, False),
        (36, 44, hot.HOT_FP64, 1e-6, hot.HOT_FLAG_FIXED_ITERS, 300, False),
        (42, 42, hot.HOT_FP64, 1e-6, R, 200000, True),
    ]
    reqs = []
    for t, (m, n, prec, tol, flags, mi, nu) in enumerate(specs):
        a = dev(workloads.gaussian_blobs(m, n, 2, rng))
        b = dev(workloads.gaussian_blobs(m, n, 3, rng))
        kw = dict(tol=tol, prec=prec, flags=flags, max_iter=mi)
        if nu:
            kw["coord_row"] = dev(workloads.grid_lines(m, rng))
            kw["coord_col"] = dev(workloads.grid_lines(n, rng))
        reqs.append((t, a, b, kw))
    srv = hot.Server(c, max_slots=6, shared=True)
    for q, (t, a, b, kw) in enumerate(reqs):
        srv.submit(a, b, t, **kw)
        if q == 2:
            time.sleep(0.02)
    assert srv.drain(300.0) == hot.HOT_OK
    got = {r["tag"]: r for r in srv.poll(16)}
    st = srv.stats()
    srv.close()
    assert len(got) == len(reqs) and st["max_shared"] >= 2
    for t, a, b, kw in reqs:
        alone, _ = c.solve(a, b, **kw)
        r = got[t]
        assert r["status"] == alone["status"] and r["status"] == hot.HOT_OK, (t, r["status"])
        for key in ("primal_obj", "dual_obj", "kkt", "kkt_abs", "feaserr", "iters", "restarts"):
            assert r[key] == alone[key], (t, key, r[key], alone[key])
