"""Pins of Algorithm 1 (plan recovery) and the marginal repair.

* Prop. 1: on an optimal (LP-exact) reduced flow, the recovered plan has the
  exact marginals and its cost equals the reduced objective, which equals the
  full OT optimum from an independent LP solver.
* At most m+n-1 positive entries come out of each bin (k,j) (the matching of
  two monotone sequences has that many pieces).
* On approximate flows the repair restores both marginals to rounding level
  while keeping every entry nonnegative.
"""
import numpy as np
import pytest

from lp_helpers import full_ot_lp, highs, rand_hist, reduced_lp


def plan_cost(m, n, src, dst, mass):
    i, j = src // n, src % n
    k, l = dst // n, dst % n
    return float(np.sum(mass * ((i - k) ** 2 + (j - l) ** 2)))


@pytest.mark.parametrize("m,n,zeros", [(3, 3, 0), (4, 4, 0.2), (3, 5, 0), (5, 4, 0.3)])
def test_prop1_on_lp_exact_flows(oracle, m, n, zeros):
    rng = np.random.default_rng(17 * m + n)
    mu1, mu2 = rand_hist(rng, m, n, zeros), rand_hist(rng, m, n, zeros)
    Ar, br, cr = reduced_lp(mu1, mu2, oracle)
    st, x, red = oracle.simplex(Ar, br, cr)
    assert st == 0
    src, dst, mass = oracle.recover(m, n, x)
    row, col = oracle.marginals(m, n, src, dst, mass)
    assert np.abs(row - mu1.ravel()).sum() <= 1e-12
    assert np.abs(col - mu2.ravel()).sum() <= 1e-12
    assert mass.min() > 0
    full, _ = highs(*full_ot_lp(mu1, mu2))
    assert abs(plan_cost(m, n, src, dst, mass) - red) <= 1e-12 * max(1, red)
    assert abs(red - full) <= 1e-9 * max(1, full)
    # per-(k,j) piece count: source (i,j) -> target (k,l) groups by (k, j)
    key = (dst // n) * n + (src % n)
    counts = np.bincount(key, minlength=m * n)
    assert counts.max() <= m + n - 1


def test_recover_matches_bruteforce_definition(oracle):
    """Alg. 1's loop on one bin equals the overlap of the two cumulative
    sequences (north-west-corner form), checked on random nonnegative rows."""
    m, n = 4, 5
    rng = np.random.default_rng(2)
    x = rng.uniform(-0.2, 1.0, size=m * m * n + m * n * n)
    x[rng.uniform(size=x.size) < 0.3] = 0
    src, dst, mass = oracle.recover(m, n, x)
    f = np.maximum(x, 0)
    for k in range(m):
        for j in range(n):
            a = np.array([f[(j * m + k) * m + i] for i in range(m)])
            b = np.array([f[m * m * n + (l * n + j) * m + k] for l in range(n)])
            P, Q = np.concatenate([[0], np.cumsum(a)]), np.concatenate([[0], np.cumsum(b)])
            sel = ((dst // n) == k) & ((src % n) == j)
            got = np.zeros((m, n))
            got[src[sel] // n, dst[sel] % n] = mass[sel]
            want = np.maximum(0, np.minimum(P[1:, None], Q[None, 1:]) -
                              np.maximum(P[:-1, None], Q[None, :-1]))
            np.testing.assert_allclose(got, want, atol=1e-15)


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_repair_restores_marginals(oracle, tol):
    m, n = 6, 6
    rng = np.random.default_rng(8)
    mu1, mu2 = rand_hist(rng, m, n, 0.1), rand_hist(rng, m, n, 0.1)
    xb, _, _, _, res = oracle.hot(mu1, mu2, tol=tol)
    src, dst, mass = oracle.recover(m, n, xb)
    row, col = oracle.marginals(m, n, src, dst, mass)
    raw = np.abs(row - mu1.ravel()).sum() + np.abs(col - mu2.ravel()).sum()
    s2, d2, w2 = oracle.repair(mu1, mu2, src, dst, mass)
    row, col = oracle.marginals(m, n, s2, d2, w2)
    assert np.abs(row - mu1.ravel()).sum() <= 1e-13
    assert np.abs(col - mu2.ravel()).sum() <= 1e-13
    assert w2.min() >= 0
    assert len(w2) <= len(mass) + 2 * m * n - 1
    cost_raw = plan_cost(m, n, src, dst, mass)
    cost_rep = plan_cost(m, n, s2, d2, w2)
    assert raw > 0
    assert abs(cost_rep - res["primal_obj"]) <= 0.05 * res["primal_obj"]
    assert cost_raw > 0
