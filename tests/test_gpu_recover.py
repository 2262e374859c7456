"""GPU plan recovery (Algorithm 1 + marginal repair) against the oracle.

* Same flows in, same plan out: the oracle's literal triple loop and repair,
  fed the GPU's exported x_bar, give the GPU plan entry for entry (dense
  comparison; the two differ only in rounding of the running totals).
* Marginals of the returned plan (summed on the host) meet mu1 and mu2 to
  1e-9 in L1 after repair; the reported errors agree with the host sums.
* Entry order: bins (k*n + j) ascending, then source, then target.
* At the 128 x 128 size, FP32 streams: marginals to 1e-6 in L1 and the plan
  cost within the solve's tolerance of <c, x_bar>.
"""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def dense(M, src, dst, mass):
    P = np.zeros((M, M))
    np.add.at(P, (src, dst), mass)
    return P


def plan_cost(n, src, dst, mass):
    i, j = src // n, src % n
    k, l = dst // n, dst % n
    return float(np.sum(mass * ((i - k) ** 2 + (j - l) ** 2)))


@pytest.mark.parametrize("m,n,tol", [(6, 6, 1e-6), (8, 8, 1e-4), (5, 9, 1e-5), (9, 4, 1e-6),
                                     (1, 12, 1e-6)])
def test_plan_matches_oracle_on_same_flows(oracle, m, n, tol):
    need_gpu()
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(workloads.seed_for(0, 100 + m * n))
    mu1 = workloads.gaussian_blobs(m, n, 2, rng)
    mu2 = workloads.masked_shape(m, n, rng) if m > 1 else workloads.white_noise(m, n, rng)
    c = ctx()
    res, sol = c.solve(dev(mu1), dev(mu2), keep=True, tol=tol)
    xb = sol.export()[0].cpu().numpy()
    src, dst, mass, err = sol.recover_plan()
    src, dst, mass = src.cpu().numpy(), dst.cpu().numpy(), mass.cpu().numpy()
    osrc, odst, omass = oracle.recover(m, n, xb)
    r0, c0 = oracle.marginals(m, n, osrc, odst, omass)
    raw = (np.abs(r0 - mu1.ravel()).sum(), np.abs(c0 - mu2.ravel()).sum())
    s2, d2, w2 = oracle.repair(mu1, mu2, osrc, odst, omass)
    M = m * n
    G, O = dense(M, src, dst, mass), dense(M, s2, d2, w2)
    assert np.abs(G - O).max() <= 1e-13 * max(1.0, O.max())
    assert mass.min() >= 0
    row, col = G.sum(1), G.sum(0)
    assert np.abs(row - mu1.ravel()).sum() <= 1e-9
    assert np.abs(col - mu2.ravel()).sum() <= 1e-9
    assert abs(err[0] - raw[0]) <= 1e-12 + 1e-9 * raw[0]
    assert abs(err[1] - raw[1]) <= 1e-12 + 1e-9 * raw[1]
    assert err[2] <= 1e-12 and err[3] <= 1e-12
    # ordering of the Algorithm 1 part: key (k*n + j, i, l) nondecreasing
    nb = len(osrc)
    i, j, k, l = src[:nb] // n, src[:nb] % n, dst[:nb] // n, dst[:nb] % n
    key = ((k * n + j) * m + i) * n + l
    assert np.all(np.diff(key) > 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_plan_at_128(oracle, prec):
    need_gpu()
    from paper_2408_00598_amd import workloads
    mu1, mu2 = workloads.pair_medium("blobs")
    n = 128
    c = ctx()
    res, sol = c.solve(dev(mu1), dev(mu2), keep=True, tol=1e-6, prec=prec)
    src, dst, mass, err = sol.recover_plan()
    src, dst, mass = src.cpu().numpy(), dst.cpu().numpy(), mass.cpu().numpy()
    M = n * n
    row = np.bincount(src, weights=mass, minlength=M)
    col = np.bincount(dst, weights=mass, minlength=M)
    assert np.abs(row - mu1.ravel()).sum() <= 1e-6
    assert np.abs(col - mu2.ravel()).sum() <= 1e-6
    assert mass.min() >= 0
    cost = plan_cost(n, src, dst, mass)
    assert abs(cost - res["primal_obj"]) <= 1e-3 * res["primal_obj"]
    assert len(mass) <= M * (2 * n - 1) + 2 * M - 1
