"""Batched solves: each problem's result is bit-identical alone and inside a
batch of uneven sizes (same kernels, fixed reduction order), and matches the
oracle to the FP64 tolerance.  Invalid inputs come back as HOT_E_INVALID."""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def test_batch_equals_alone_bitwise():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(12, sides=(8, 12, 16, 24))
    c = ctx()
    dp = [(dev(a), dev(b)) for a, b in pairs]
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        batch = c.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec)
        for (a, b), rb in zip(dp, batch):
            ra, _ = c.solve(a, b, tol=1e-5, max_iter=200000, prec=prec)
            for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
                assert ra[key] == rb[key], (key, ra[key], rb[key])


def test_fused_and_split_slab_kernels_bitwise(monkeypatch):
    """One slab kernel for every pass kind and the split plain / check-restart
    kernels do the same arithmetic in the same order: identical results and
    states, for block and wave-per-slab families, both precisions."""
    need_gpu()
    import torch
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(40, sides=(16, 24, 32, 48, 96, 130))
    # enough small slabs (side <= 48) for the launch to take the wave-per-slab pass
    assert sum(2 * a.shape[0] for a, _ in pairs if a.shape[0] <= 48) >= 1024
    dp = [(dev(a), dev(b)) for a, b in pairs]
    ctxs = []
    for fuse in ("0", "1"):
        monkeypatch.setenv("HOT_FUSE", fuse)
        ctxs.append(hot.Context(0))
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        rs = [c.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec) for c in ctxs]
        for ra, rb in zip(*rs):
            for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
                assert ra[key] == rb[key], (prec, key, ra[key], rb[key])
        rng = np.random.default_rng(workloads.seed_for(0, 130))
        a = dev(workloads.gaussian_blobs(130, 130, 3, rng))
        b = dev(workloads.gaussian_blobs(130, 130, 3, rng))
        outs = []
        for c in ctxs:
            r, sol = c.solve(a, b, keep=True, max_iter=137, prec=prec,
                             flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_FIXED_ITERS)
            outs.append((r, [t.cpu() for t in sol.export()]))
        assert outs[0][0]["primal_obj"] == outs[1][0]["primal_obj"]
        for t0, t1 in zip(outs[0][1], outs[1][1]):
            assert torch.equal(t0, t1)


@pytest.mark.parametrize("variant", ["sigma_update", "nonuniform", "both"])
def test_fused_and_split_variants_bitwise(monkeypatch, variant):
    """The same for sigma re-balancing at restarts and non-uniform bins (the
    variants whose check and restart rows carry extra work)."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(0, 77))
    m, n = 40, 72
    a = dev(workloads.gaussian_blobs(m, n, 3, rng))
    b = dev(workloads.gaussian_blobs(m, n, 3, rng))
    kw = dict(tol=1e-6, max_iter=20000)
    if variant != "nonuniform":
        kw["flags"] = hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE
    if variant != "sigma_update":
        kw["coord_row"] = dev(workloads.grid_lines(m, rng))
        kw["coord_col"] = dev(workloads.grid_lines(n, rng))
    res = []
    for fuse in ("0", "1"):
        monkeypatch.setenv("HOT_FUSE", fuse)
        c = hot.Context(0)
        res.append([c.solve(a, b, prec=p, **kw)[0] for p in (hot.HOT_FP64, hot.HOT_FP32_STREAM)])
    # (converged or stopped at max_iter alike: restarts and check passes ran)
    assert res[0][0]["restarts"] > 0
    for ra, rb in zip(*res):
        for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
            assert ra[key] == rb[key], (variant, key, ra[key], rb[key])


def test_row_grouping_bitwise(monkeypatch):
    """Solve waves of one, three or four slabs and reduce blocks of as many
    slots compute every slab's values and every slot's partials the same
    way: identical results (the default groups four for launches with many
    row blocks)."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(8, sides=(16, 40, 72, 130))
    dp = [(dev(a), dev(b)) for a, b in pairs]
    ctxs = []
    for spw, rq in (("1", "1"), ("4", "4"), ("3", "2")):
        monkeypatch.setenv("HOT_ROW_GROUP", spw)
        monkeypatch.setenv("HOT_REDUCE_GROUP", rq)
        ctxs.append(hot.Context(0))
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        rs = [c.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec) for c in ctxs]
        for other in rs[1:]:
            for ra, rb in zip(rs[0], other):
                for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
                    assert ra[key] == rb[key], (prec, key, ra[key], rb[key])


def test_batch_matches_oracle(oracle):
    need_gpu()
    from paper_2408_00598_amd import workloads
    pairs = workloads.batch_pairs(6, sides=(6, 10, 14))
    c = ctx()
    res = c.batch_solve([(dev(a), dev(b)) for a, b in pairs], tol=1e-6, max_iter=200000)
    for (a, b), r in zip(pairs, res):
        _, _, _, _, o = oracle.hot(a, b, tol=1e-6, max_iter=200000)
        assert r["status"] == 0 and o["converged"] == 1
        assert r["iters"] == o["iters"]
        assert abs(r["primal_obj"] - o["primal_obj"]) <= 1e-6 * abs(o["primal_obj"])


def test_rectangular_and_degenerate_shapes(oracle):
    need_gpu()
    rng = np.random.default_rng(5)
    c = ctx()
    for m, n in [(1, 1), (1, 2), (2, 1), (3, 17), (17, 3), (4, 64)]:
        mu1 = rng.uniform(0.1, 1, (m, n)); mu1 /= mu1.sum()
        mu2 = rng.uniform(0.1, 1, (m, n)); mu2 /= mu2.sum()
        r, _ = c.solve(dev(mu1), dev(mu2), tol=1e-7, max_iter=400000)
        _, _, _, _, o = oracle.hot(mu1, mu2, tol=1e-7, max_iter=400000)
        assert r["status"] == 0 and o["converged"] == 1
        assert abs(r["primal_obj"] - o["primal_obj"]) <= 1e-6 * max(abs(o["primal_obj"]), 1e-9)


def test_invalid_inputs_rejected():
    need_gpu()
    from paper_2408_00598_amd import hot
    c = ctx()
    good = np.full((4, 4), 1 / 16)
    bad_neg = good.copy(); bad_neg[0, 0] = -1e-3; bad_neg[0, 1] += 1e-3
    bad_nan = good.copy(); bad_nan[1, 1] = np.nan
    bad_mass = good * 1.01
    for bad in (bad_neg, bad_nan, bad_mass):
        r, _ = c.solve(dev(good), dev(bad), tol=1e-6, raise_on_error=False)
        assert r["return_status"] == hot.HOT_E_INVALID
        assert c.last_error()
    r, _ = c.solve(dev(good), dev(good), tol=0.0, raise_on_error=False)
    assert r["return_status"] == hot.HOT_E_INVALID
    r, _ = c.solve(dev(good), dev(good), tol=1e-6, max_iter=0, raise_on_error=False)
    assert r["return_status"] == hot.HOT_E_INVALID


def test_not_converged_reports_last_iterate():
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    mu1, mu2 = workloads.pair_small()
    c = ctx()
    r, _ = c.solve(dev(mu1), dev(mu2), tol=1e-9, max_iter=35, raise_on_error=False)
    assert r["return_status"] == hot.HOT_E_NOT_CONVERGED
    assert r["iters"] == 35 and r["kkt"] > 1e-9 and np.isfinite(r["primal_obj"])


def test_zero_mass_bins(oracle):
    need_gpu()
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(workloads.seed_for(0, 777))
    mu1, mu2 = workloads.masked_shape(16, 16, rng), workloads.masked_shape(16, 16, rng)
    c = ctx()
    r, sol = c.solve(dev(mu1), dev(mu2), keep=True, tol=1e-6)
    _, _, _, _, o = oracle.hot(mu1, mu2, tol=1e-6)
    assert r["status"] == 0
    assert abs(r["primal_obj"] - o["primal_obj"]) <= 1e-6 * abs(o["primal_obj"])
    src, dst, mass, err = sol.recover_plan()
    assert err[2] <= 1e-12 and err[3] <= 1e-12


def test_batch_with_early_finishers_equals_alone():
    """Most problems of the batch stop after a few checks (identical source and
    target), so the launch tables are rebuilt for the remaining ones while they
    iterate; every result still equals its solo solve bit for bit."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(77)
    slow = workloads.batch_pairs(4, sides=(12, 16))
    fast = []
    for n in (8, 10, 12, 14, 16, 20, 8, 10):
        h = rng.uniform(0.1, 1, (n, n))
        h /= h.sum()
        fast.append((h, h.copy()))
    pairs = fast[:4] + slow[:2] + fast[4:] + slow[2:]
    c = ctx()
    dp = [(dev(a), dev(b)) for a, b in pairs]
    batch = c.batch_solve(dp, tol=1e-6, max_iter=200000)
    iters = [r["iters"] for r in batch]
    assert max(iters) > 4 * min(iters)
    for (a, b), rb in zip(dp, batch):
        ra, _ = c.solve(a, b, tol=1e-6, max_iter=200000)
        for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status"):
            assert ra[key] == rb[key], (key, ra[key], rb[key])


def test_batch_consecutive_compactions_equal_alone():
    """Problems of each group stop on consecutive graphs (fixed iteration
    counts 15, 35, 55 and 200), so the launch tables are rebuilt on three
    consecutive polls while the previous upload may still be queued; every
    result equals its solo solve bit for bit."""
    need_gpu()
    from paper_2408_00598_amd import hot
    rng = np.random.default_rng(91)
    per_group = [15, 15, 15, 15, 35, 35, 55, 200]
    pairs, iters = [], []
    for p in range(16):  # equal sizes: the two groups take every other pair
        a, b = rng.uniform(0.1, 1, (12, 12)), rng.uniform(0.1, 1, (12, 12))
        K = per_group[p // 2]
        pairs.append((dev(a / a.sum()), dev(b / b.sum()), {"max_iter": K}))
        iters.append(K)
    c = ctx()
    batch = c.batch_solve(pairs, flags=hot.HOT_FLAG_FIXED_ITERS)
    for (a, b, kw), rb, K in zip(pairs, batch, iters):
        ra, _ = c.solve(a, b, max_iter=K, flags=hot.HOT_FLAG_FIXED_ITERS)
        assert rb["iters"] == K
        for key in ("primal_obj", "dual_obj", "kkt", "feaserr", "iters", "status"):
            assert ra[key] == rb[key], (key, ra[key], rb[key])


def test_graph_replays_equal_direct_launches_bitwise(monkeypatch):
    """Iterations run as captured graphs, replayed many times with host reads
    of the control blocks and unrelated eager device work in between, give
    the same results and states as the same iterations launched directly
    (HOT_NO_GRAPH=1): batch and single-pair paths, both precisions, and a
    second graph solve on the same context after eager work."""
    need_gpu()
    import torch
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(24, sides=(16, 24, 32, 64, 96))
    dp = [(dev(a), dev(b)) for a, b in pairs]
    rng = np.random.default_rng(workloads.seed_for(1, 72))
    a = dev(workloads.gaussian_blobs(72, 72, 3, rng))
    b = dev(workloads.gaussian_blobs(72, 72, 3, rng))
    monkeypatch.setenv("HOT_NO_GRAPH", "1")
    direct = hot.Context(0)
    monkeypatch.delenv("HOT_NO_GRAPH")
    graph = hot.Context(0)
    keys = ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status")
    side = torch.arange(1 << 20, device="cuda:0", dtype=torch.float64)
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        monkeypatch.setenv("HOT_NO_GRAPH", "1")
        want = direct.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec)
        rw, sw = direct.solve(a, b, keep=True, max_iter=300, prec=prec,
                              flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_FIXED_ITERS)
        want_state = [t.cpu() for t in sw.export()]
        monkeypatch.delenv("HOT_NO_GRAPH")
        for rep in range(2):
            got = graph.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec)
            for ra, rb in zip(want, got):
                assert rb["iters"] > 0
                for key in keys:
                    assert ra[key] == rb[key], (prec, rep, key, ra[key], rb[key])
            rg, sg = graph.solve(a, b, keep=True, max_iter=300, prec=prec,
                                 flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_FIXED_ITERS)
            for key in keys:
                assert rw[key] == rg[key], (prec, rep, key, rw[key], rg[key])
            for t0, t1 in zip(want_state, sg.export()):
                assert torch.equal(t0, t1.cpu())
            # eager device work and a synchronisation between the two rounds
            assert float((side * 2.0).sum().item()) == float((1 << 20) * ((1 << 20) - 1))
            torch.cuda.synchronize()


def test_solve_load_order_bitwise(monkeypatch):
    """The solve issuing its decision-free loads before the decision
    (HOT_SOLVE_PRE=1) or after it (0) computes the same values: identical
    results and states, batch (tiles and several slabs per wave) and a
    rectangular single pair, both precisions."""
    need_gpu()
    import torch
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(20, sides=(8, 24, 40, 72, 130))
    dp = [(dev(a), dev(b)) for a, b in pairs]
    rng = np.random.default_rng(workloads.seed_for(2, 70))
    a = rng.uniform(0.05, 1, (70, 45)); a /= a.sum()
    b = rng.uniform(0.05, 1, (70, 45)); b /= b.sum()
    a, b = dev(a), dev(b)
    ctxs = []
    for pre in ("0", "1"):
        monkeypatch.setenv("HOT_SOLVE_PRE", pre)
        ctxs.append(hot.Context(0))
    keys = ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "status")
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        rs = [c.batch_solve(dp, tol=1e-5, max_iter=200000, prec=prec) for c in ctxs]
        for ra, rb in zip(*rs):
            for key in keys:
                assert ra[key] == rb[key], (prec, key, ra[key], rb[key])
        outs = []
        for c in ctxs:
            r, sol = c.solve(a, b, keep=True, max_iter=151, prec=prec,
                             flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_FIXED_ITERS)
            outs.append((r, [t.cpu() for t in sol.export()]))
        for key in keys:
            assert outs[0][0][key] == outs[1][0][key], (prec, key)
        for t0, t1 in zip(outs[0][1], outs[1][1]):
            assert torch.equal(t0, t1)
