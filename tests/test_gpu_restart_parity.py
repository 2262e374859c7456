"""Parity through restarts at the benchmarked sizes (Alg. 2 Steps 1-4 with the
restart rule, Prop. 3), against the oracle's own operators.

The oracle cannot run these sizes to a restart in test time, so each case
takes the GPU iterate after K updates of a restarted solve (at least two
restarts behind it, the epoch's Halpern anchor a buffer of its own) and
recomputes from it, entry by entry, with the oracle's A, Prop. 3 solve
(W-hat form) and A^T:
  * y_bar^K = (A A^T)^{-1} (b/sigma - A(s^K - c));
  * the next update s^{K+1} = lam s^0 + (1 - lam)|s^K - 2 g^K|,
    g^K = c - A^T y_bar^K, lam = 1/(k+2) with k the epoch counter
    (taken from a second solve stopped one update later);
  * the anchor itself, s^0 = max(s^r - g^r, g^r), from the state s^r of the
    check that restarted the epoch (a third solve stopped at that check).
96 x 96 and 128 x 128 run in the 256-pair batch's tuned launch shape.
"""
import numpy as np
import pytest

from gpu_helpers import dev, need_gpu

pytestmark = pytest.mark.gpu

T = 10
TUNED = {"HOT_ITEM_ELEMS": "8192", "HOT_UNROLL": "2", "HOT_VPL_TARGET": "2"}


def close(a, b, tol, floor):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max()) <= tol * max(float(np.abs(b).max()), floor)


def run(c, d1, d2, K, prec):
    res, sol = c.solve(d1, d2, keep=True, tol=1e-14, max_iter=K, prec=prec)
    assert res["iters"] == K and res["status"] == 4  # stopped by max_iter
    return res, sol


def restart_case(oracle, c, mu1, mu2, prec, K0):
    from paper_2408_00598_amd import hot
    m, n = mu1.shape
    d1, d2 = dev(mu1), dev(mu2)
    fp32 = prec == hot.HOT_FP32_STREAM
    K = K0
    for _ in range(40):
        res, sol = run(c, d1, d2, K, prec)
        s0_d, info = sol.anchor()
        if res["restarts"] >= 2 and info["k"] % T != 0 and info["anchor"] == 2:
            break
        sol.free()
        K = 2 * K if res["restarts"] < 2 else K + 1
    else:
        pytest.fail("no iterate with two restarts behind it")
    k, lam, sigma = info["k"], info["lam"], info["sigma"]
    assert lam == 1.0 / (k + 2)
    print(f"case {m}x{n} prec={prec} K={K} restarts={res['restarts']} k={k}", flush=True)
    _, yb_d, _, s_d = sol.export()
    yK, sK = yb_d.cpu().numpy(), s_d.cpu().numpy()
    s0 = s0_d.cpu().numpy()
    sol.free()
    del yb_d, s_d, s0_d
    # one update later
    r1, sol1 = run(c, d1, d2, K + 1, prec)
    assert r1["restarts"] == res["restarts"]
    s_next = sol1.export()[3].cpu().numpy()
    sol1.free()
    # the check that restarted the epoch: K - k updates ago, minus the restart
    r_at = K - k - 1
    rr, solr = run(c, d1, d2, r_at, prec)
    assert rr["restarts"] == res["restarts"] - 1
    _, yr_d, _, sr_d = solr.export()
    yr, sr = yr_d.cpu().numpy(), sr_d.cpu().numpy()
    solr.free()
    del yr_d, sr_d

    cst = oracle.cost(m, n)
    b = oracle.bvec(mu1, mu2)
    assert abs(sigma - np.linalg.norm(b) / np.linalg.norm(cst)) <= 1e-12 * sigma
    # Step 1 at K: the GPU's y_bar from the oracle's A and Prop. 3
    y_or = oracle.solve_aat(m, n, b / sigma - oracle.A(m, n, sK - cst))
    assert close(yK, y_or, 1e-9, 1.0)
    # Steps 2-4 at K with the separate anchor
    g = cst - oracle.AT(m, n, yK)
    want = lam * s0 + (1.0 - lam) * np.abs(sK - 2.0 * g)
    assert close(s_next, want, 2e-7 if fp32 else 1e-10, 1e-3)
    del want, g
    # the restart pass: the anchor is s_bar = max(s - g, g) at the restarting check
    gr = cst - oracle.AT(m, n, yr)
    sbar = np.maximum(sr - gr, gr)
    assert close(s0, sbar, 2e-7 if fp32 else 1e-12, 1e-3)


@pytest.mark.parametrize("side", [96, 128])
@pytest.mark.parametrize("prec_name", ["HOT_FP32_STREAM", "HOT_FP64"])
def test_restart_parity_batch_sides(monkeypatch, oracle, side, prec_name):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    for kv in TUNED.items():
        monkeypatch.setenv(*kv)
    rng = np.random.default_rng(workloads.seed_for(3, side))
    mu1, mu2 = workloads.gaussian_blobs(side, side, 4, rng), workloads.gaussian_blobs(side, side, 4, rng)
    restart_case(oracle, hot.Context(0), mu1, mu2, getattr(hot, prec_name), 200)


@pytest.mark.parametrize("prec_name", ["HOT_FP32_STREAM", "HOT_FP64"])
def test_restart_parity_192_noise(oracle, prec_name):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    rng = np.random.default_rng(workloads.seed_for(4, 192))
    mu1, mu2 = workloads.white_noise(192, 192, rng), workloads.white_noise(192, 192, rng)
    restart_case(oracle, hot.Context(0), mu1, mu2, getattr(hot, prec_name), 200)


@pytest.mark.parametrize("prec_name", ["HOT_FP32_STREAM", "HOT_FP64"])
def test_restart_parity_512(oracle, prec_name):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    mu1, mu2 = workloads.pair_large(0)
    restart_case(oracle, hot.Context(0), mu1, mu2, getattr(hot, prec_name), 200)
