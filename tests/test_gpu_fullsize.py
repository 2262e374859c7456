"""Parity at the benchmark's full sizes, in its launch configuration.

The oracle cannot iterate at 512 x 512 in test time (N = 2.7e8 flows), so the
full-size checks take the GPU iterate after K fixed iterations and recompute
one whole step from it with the oracle's own operators: R = b/sigma - A(s - c)
(oracle A), y_bar from the oracle's Prop. 3 solve, x_bar = sigma(s - g) with
the oracle's A^T.  Every entry is compared.  Converged solves at full size
are checked by properties that hold at any size: A x_bar = b to roundoff
(the s-form keeps it at every iterate), the stopping test, FP32 streams
against FP64, and a repaired plan that meets the marginals and costs at
least the marginal lower bound.  The 256-pair batch is solved whole and
sampled pairs are re-solved by the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def close(a, b, tol, floor):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max()) <= tol * max(float(np.abs(b).max()), floor)


def one_step_against_oracle(oracle, c, mu1, mu2, K, prec, tol_y=1e-9):
    from paper_2408_00598_amd import hot
    m, n = mu1.shape
    res, sol = c.solve(dev(mu1), dev(mu2), keep=True, max_iter=K, prec=prec,
                       flags=hot.HOT_FLAG_FIXED_ITERS)
    xb_d, yb_d, _, s_d = sol.export()
    yb = yb_d.cpu().numpy()
    s = s_d.cpu().numpy()
    del yb_d, s_d
    assert res["iters"] == K and np.isfinite(s).all() and s.min() >= 0.0
    cst = oracle.cost(m, n)
    b = oracle.bvec(mu1, mu2)
    sigma = np.linalg.norm(b) / np.linalg.norm(cst)
    assert abs(res["sigma"] - sigma) <= 1e-12 * sigma
    t = s - cst
    del s, cst
    R = b / sigma - oracle.A(m, n, t)
    y_or = oracle.solve_aat(m, n, R)
    assert close(yb, y_or, tol_y, 1.0)
    t += oracle.AT(m, n, y_or)
    t *= sigma  # x_bar = sigma (s - c + A^T y_bar)
    xb = xb_d.cpu().numpy()
    del xb_d
    assert close(xb, t, 1e-8, 1e-3)
    sol.free()


@pytest.mark.parametrize("prec_name", ["HOT_FP32_STREAM", "HOT_FP64"])
def test_512_step_against_oracle_operators(oracle, prec_name):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    mu1, mu2 = workloads.pair_large(0)
    c = ctx()
    one_step_against_oracle(oracle, c, mu1, mu2, 30, getattr(hot, prec_name))


@pytest.mark.parametrize("m,n", [(1024, 48), (48, 1024)])
def test_rectangular_at_scale_step_against_oracle(oracle, m, n):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(2, m + n))
    mu1, mu2 = workloads.mixture_with_cauchy(m, n, rng), workloads.mixture_with_cauchy(m, n, rng)
    c = ctx()
    one_step_against_oracle(oracle, c, mu1, mu2, 12, hot.HOT_FP32_STREAM)


def test_512_aat_solve_against_oracle(oracle):
    need_gpu()
    m = n = 512
    rng = np.random.default_rng(512)
    R = rng.standard_normal(3 * m * n - 1)
    y = ctx().aat_solve(m, n, dev(R)).cpu().numpy()
    assert close(y, oracle.solve_aat(m, n, R), 1e-12, 1e-300)


def test_512_converged_properties(oracle):
    """configs' 512 x 512 pair at rel KKT 1e-4, FP32 streams (tuned as the
    benchmark tunes) against FP64, with the recovered plan."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    mu1, mu2 = workloads.pair_large(0)
    n = 512
    c = ctx()
    c.autotune([(dev(mu1), dev(mu2))], iters=30, prec=hot.HOT_FP32_STREAM)
    out = {}
    for prec in (hot.HOT_FP32_STREAM, hot.HOT_FP64):
        r, sol = c.solve(dev(mu1), dev(mu2), tol=1e-4, max_iter=50000, prec=prec, keep=True)
        assert r["status"] == 0 and r["kkt"] <= 1e-4
        assert r["res_primal"] <= 1e-12
        src, dst, mass, err = sol.recover_plan()
        assert err[2] <= 1e-9 and err[3] <= 1e-9
        si, sj = np.divmod(src.cpu().numpy(), n)
        di, dj = np.divmod(dst.cpu().numpy(), n)
        out[prec] = (r, float((((si - di) ** 2 + (sj - dj) ** 2) * mass.cpu().numpy()).sum()))
        sol.free()
    (r32, p32), (r64, p64) = out[hot.HOT_FP32_STREAM], out[hot.HOT_FP64]
    assert abs(r32["primal_obj"] - r64["primal_obj"]) <= 1e-4 * abs(r64["primal_obj"])
    lb = oracle.w2_1d(mu1.sum(1), mu2.sum(1)) + oracle.w2_1d(mu1.sum(0), mu2.sum(0))
    # a feasible plan costs at least the optimum, which is at least lb
    assert p32 >= lb * (1 - 1e-12) and p64 >= lb * (1 - 1e-12)


def test_1024_max_side_fixed_iterations():
    """Largest side the library accepts: FP32 streams against FP64 after
    fixed iterations (same kernels, the state rounded to FP32)."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(2, 1024))
    mu1, mu2 = workloads.mixture_with_cauchy(1024, 1024, rng), \
        workloads.mixture_with_cauchy(1024, 1024, rng)
    c = ctx()
    r = {}
    for prec in (hot.HOT_FP32_STREAM, hot.HOT_FP64):
        r[prec], _ = c.solve(dev(mu1), dev(mu2), max_iter=6, prec=prec,
                             flags=hot.HOT_FLAG_FIXED_ITERS)
        assert r[prec]["iters"] == 6 and r[prec]["res_primal"] <= 1e-12
    a, b = r[hot.HOT_FP32_STREAM], r[hot.HOT_FP64]
    assert abs(a["primal_obj"] - b["primal_obj"]) <= 1e-5 * abs(b["primal_obj"])


@pytest.mark.parametrize("prec_name", ["HOT_FP64", "HOT_FP32_STREAM"])
def test_batch256_sampled_against_oracle(oracle, prec_name):
    """The benchmark's batch (256 pairs, sides 32..128, half noise), tuned
    and launched as the benchmark does; sampled pairs re-solved by the oracle.

    FP64: the first three 32 x 32 pairs and the first 48 x 48 pair stop at
    the oracle's iteration with its objective (1e-6).  FP32 streams stop at a
    nearby but different iterate, and at rel KKT 1e-4 the objective is only
    determined to about 1e-2 (the oracle's own value at 1e-4 is 0.05% to 3%
    off the optimum on these 32 x 32 pairs), so the FP32 bar at this
    tolerance is the oracle's own error: |obj32 - opt| <= 2 |obj_or - opt|
    + 1e-4 opt, with opt the oracle at 1e-6.  The 1e-4 objective bar for
    FP32 streams at a tolerance that fixes the objective is
    test_converged_solve_fp32_streams."""
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    prec = getattr(hot, prec_name)
    pairs = workloads.batch_pairs(256)
    c = ctx()
    dp = [(dev(a), dev(b)) for a, b in pairs]
    c.autotune(dp, iters=30, prec=prec)
    res = c.batch_solve(dp, tol=1e-4, max_iter=100000, prec=prec)
    for r in res:
        assert r["status"] == 0 and r["kkt"] <= 1e-4 and r["res_primal"] <= 1e-12
    sides = [a.shape[0] for a, _ in pairs]
    sample = [i for i, s in enumerate(sides) if s == 32][:3]
    if prec == hot.HOT_FP64:
        sample.append(sides.index(48))
    for i in sample:
        o = oracle.hot(*pairs[i], tol=1e-4, max_iter=100000)[4]
        assert o["converged"] == 1
        if prec == hot.HOT_FP64:
            assert res[i]["iters"] == o["iters"] and res[i]["restarts"] == o["restarts"]
            assert abs(res[i]["primal_obj"] - o["primal_obj"]) <= 1e-6 * abs(o["primal_obj"])
        else:
            opt = oracle.hot(*pairs[i], tol=1e-6, max_iter=200000)[4]["primal_obj"]
            band = 2 * abs(o["primal_obj"] - opt) + 1e-4 * abs(opt)
            assert abs(res[i]["primal_obj"] - opt) <= band, (i, res[i]["primal_obj"], opt, band)
