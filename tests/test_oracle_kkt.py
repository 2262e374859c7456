"""Pins of the oracle's stopping rule and restart rule.

* eq. kkt_res (Sec. 4, experimental setup): the three normalised residuals
  and their maximum, and the feasibility error of Sec. 4.1, recomputed here
  with numpy from the Kronecker-product A of def:A1A2A3 / def:A4 and from b
  and c built from their definitions (eq. Mat:A&b, eq. def:c), on arbitrary
  iterates (where every residual is far from zero, so a wrong denominator
  shows) and along the oracle's own trajectories.
* The restart rule (check every T = 10 iterations of an epoch, fixed-point
  residual r = ||s - shat||, restart when r <= 0.2 r_start, or when
  r <= 0.8 r_start and r grew since the previous check): the residuals of the
  first epoch are recomputed from restart-free runs (and, at k = 0, from a
  dense numpy solve of Step 1), the first restart must land where the rule
  puts it, and every later decision recorded by the oracle must follow the
  rule applied to the recorded residuals.
"""
import numpy as np
import pytest

from lp_helpers import kron_A, rand_hist


def b_of(mu1, mu2):
    """b = [0_M; vec(mu1); Ibar vec(mu2)], images vectorised with the row index
    fastest (the order the Kronecker forms of A3 and A4 imply)."""
    M = mu1.size
    return np.concatenate([np.zeros(M), mu1.T.ravel(), mu2.T.ravel()[:-1]])


def c_of(m, n):
    """c = [c1; c2]: c1_{i,k,j} = (k - i)^2 at (j m + k) m + i and
    c2_{k,j,l} = (j - l)^2 at m m n + (l n + j) m + k."""
    i = np.arange(m)
    j = np.arange(n)
    c1 = np.broadcast_to((i[None, :, None] - i[None, None, :]) ** 2,
                         (n, m, m)).astype(float)          # [j][k][i]: (k - i)^2
    c2 = np.broadcast_to((j[:, None, None] - j[None, :, None]) ** 2,
                         (n, n, m)).astype(float)          # [l][j][k]: (j - l)^2
    return np.concatenate([c1.ravel(), c2.ravel()])


def kkt_numpy(A, b, c, x, y, z):
    rd = np.linalg.norm(A.T @ y + z - c) / (1 + np.linalg.norm(c))
    rc = np.linalg.norm(np.minimum(x, z)) / (1 + np.linalg.norm(x) + np.linalg.norm(z))
    rp = np.linalg.norm(A @ x - b) / (1 + np.linalg.norm(b))
    fe = max(np.linalg.norm(np.minimum(x, 0.0)) / (1 + np.linalg.norm(x)), rp)
    return {"res_dual": rd, "res_comp": rc, "res_primal": rp, "kkt": max(rd, rc, rp),
            "feaserr": fe, "primal_obj": c @ x, "dual_obj": b @ y}


def close(a, b, rtol=1e-12, atol=0.0):
    return abs(a - b) <= rtol * max(abs(a), abs(b)) + atol


@pytest.mark.parametrize("m,n", [(3, 4), (4, 4), (5, 3)])
def test_b_and_c_match_definitions(oracle, m, n):
    rng = np.random.default_rng(m * 10 + n)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    assert np.array_equal(oracle.bvec(mu1, mu2), b_of(mu1, mu2))
    assert np.array_equal(oracle.cost(m, n), c_of(m, n))


@pytest.mark.parametrize("m,n,seed", [(3, 4, 1), (4, 5, 2), (5, 5, 3)])
def test_kkt_res_on_arbitrary_iterates(oracle, m, n, seed):
    """Arbitrary (x, y, z) with negative entries in x: every residual is of
    order one, so the normalisations (1 + ||c||, 1 + ||x|| + ||z||, the
    reduced b with 3M - 1 rows) are each visible."""
    rng = np.random.default_rng(seed)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    A, b, c = kron_A(m, n), b_of(mu1, mu2), c_of(m, n)
    N, M3 = A.shape[1], A.shape[0]
    for trial in range(4):
        x = rng.normal(size=N) * 10.0 ** rng.integers(-3, 1)
        y = rng.normal(size=M3) * 10.0 ** rng.integers(-1, 2)
        z = np.abs(rng.normal(size=N)) * 10.0 ** rng.integers(-1, 2)
        ref = kkt_numpy(A, b, c, x, y, z)
        got = oracle.kkt(mu1, mu2, x, y, z)
        for key in ("res_dual", "res_comp", "res_primal", "kkt", "feaserr",
                    "primal_obj", "dual_obj"):
            assert close(got[key], ref[key]), (key, got[key], ref[key])
        # the three residuals differ, so the max picks one of them
        assert got["kkt"] in (got["res_dual"], got["res_comp"], got["res_primal"])


@pytest.mark.parametrize("K", [1, 7, 30])
def test_kkt_res_along_trajectory(oracle, K):
    """What the oracle reports after K fixed updates is eq. kkt_res of the
    iterate it exports."""
    m, n = 4, 5
    rng = np.random.default_rng(40 + K)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    A, b, c = kron_A(m, n), b_of(mu1, mu2), c_of(m, n)
    xb, yb, zb, _, res = oracle.hot(mu1, mu2, fixed_iters=K)
    ref = kkt_numpy(A, b, c, xb, yb, zb)
    for key in ("res_dual", "res_comp", "kkt", "primal_obj", "dual_obj"):
        assert close(res[key], ref[key]), (key, res[key], ref[key])
    # A x_bar = b holds to rounding at every iterate: compare at that level
    assert res["res_primal"] <= 1e-14 and ref["res_primal"] <= 1e-14
    assert res["kkt"] == max(res["res_dual"], res["res_comp"], res["res_primal"])
    assert close(res["feaserr"], ref["feaserr"], atol=1e-15)


def test_kkt_res_at_convergence(oracle):
    m, n = 5, 4
    rng = np.random.default_rng(77)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    A, b, c = kron_A(m, n), b_of(mu1, mu2), c_of(m, n)
    for tol in (1e-4, 1e-6):
        xb, yb, zb, _, res = oracle.hot(mu1, mu2, tol=tol, max_iter=400000)
        ref = kkt_numpy(A, b, c, xb, yb, zb)
        assert res["converged"] == 1
        assert ref["kkt"] <= tol
        assert close(res["kkt"], ref["kkt"], rtol=1e-10, atol=1e-15)
        assert close(res["res_dual"], ref["res_dual"], rtol=1e-10)
        assert close(res["res_comp"], ref["res_comp"], rtol=1e-10)


def _step1_numpy(A, b, c, sigma):
    """w_bar^0 from w^0 = 0 by Alg. 2 Steps 1-3 with a dense solve."""
    y = np.linalg.solve(A @ A.T, b / sigma + A @ c)
    x = sigma * (A.T @ y - c)
    z = np.maximum(0.0, c - A.T @ y - x / sigma)
    return x, z


@pytest.mark.parametrize("m,n,seed", [(4, 5, 5), (5, 5, 6), (3, 6, 7)])
def test_restart_rule_trace(oracle, m, n, seed):
    rng = np.random.default_rng(seed)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    T = 10
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-9, max_iter=200000, check_every=T,
                                 trace=100000)
    tr = res["trace"]
    assert res["converged"] == 1 and res["restarts"] >= 2
    assert len(tr) == res["ntrace"] and tr[:, 3].sum() == res["restarts"]
    sigma = res["sigma"]
    # --- first epoch: residuals recomputed from restart-free runs ----------
    A, b, c = kron_A(m, n), b_of(mu1, mu2), c_of(m, n)
    x0, z0 = _step1_numpy(A, b, c, sigma)
    r_ref = {0: 2.0 * np.linalg.norm(x0 / sigma + z0)}   # s^0 = 0
    first = int(np.flatnonzero(tr[:, 3] == 1)[0])
    for row in tr[1:first + 1]:
        k = int(row[1])
        xb, _, zb, s, r0 = oracle.hot(mu1, mu2, fixed_iters=k, restart=False)
        assert r0["sigma"] == sigma
        r_ref[k] = 2.0 * np.linalg.norm(s - (xb / sigma + zb))
    for row in tr[:first + 1]:
        k = int(row[1])
        assert int(row[0]) == k  # no restart yet: the iteration count is k
        assert close(row[2], r_ref[k], rtol=1e-9), (k, row[2], r_ref[k])
    # the rule with the stated constants, applied to the recomputed residuals
    r_start = r_ref[0]
    r_prev = r_start
    want = None
    for k in range(T, 100000, T):
        if k not in r_ref:
            break
        r = r_ref[k]
        if r <= 0.2 * r_start or (r <= 0.8 * r_start and r > r_prev):
            want = k
            break
        r_prev = r
    assert want is not None and int(tr[first, 1]) == want
    # --- every recorded decision follows the rule --------------------------
    r_start = r_prev = None
    for q, (it, k, r, flag) in enumerate(tr):
        k = int(k)
        assert k % T == 0 or q == len(tr) - 1
        if k == 0:
            assert flag == 0
            r_start = r_prev = r
            continue
        rule = r <= 0.2 * r_start or (r <= 0.8 * r_start and r > r_prev)
        if q == len(tr) - 1:
            break  # the converging check stops instead
        assert bool(flag) == rule, (q, it, k, r, r_start, r_prev)
        if flag:
            # the restart counts as an iteration; the next check is k = 0
            assert tr[q + 1, 1] == 0 and tr[q + 1, 0] == it + 1
        else:
            r_prev = r
