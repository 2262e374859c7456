"""Oracle pins for non-uniform bins: a grid whose rows sit at u_i and columns
at v_j (the K-means grid lines of the color-transfer application, Sec. 4.2).
The reduced model only changes through c; A and b are the same.

Pins: HiGHS on the full OT LP with the Euclidean cost of the non-uniform
bins; the 1-D quantile closed form at arbitrary sorted positions; the
separable closed form; scaling of the coordinates; the uniform grid given
explicitly equals the default path bit for bit.
"""
import numpy as np
import pytest

from lp_helpers import (full_ot_lp_xy, highs, kron_A, rand_hist, w2_1d_positions)


def coords(rng, L, spread=3.0, sort=True):
    x = np.cumsum(rng.uniform(0.2, spread, L)) + rng.uniform(-5, 5)
    if not sort:
        x = rng.permutation(x)
    return x


@pytest.mark.parametrize("m,n,sort", [(3, 4, True), (4, 3, True), (4, 4, False), (2, 5, True)])
def test_nonuniform_matches_full_lp(oracle, m, n, sort):
    rng = np.random.default_rng(100 * m + n)
    mu1, mu2 = rand_hist(rng, m, n, 0.15), rand_hist(rng, m, n, 0.15)
    u, v = coords(rng, m, sort=sort), coords(rng, n, sort=sort)
    Aeq, beq, c = full_ot_lp_xy(mu1, mu2, u, v)
    opt, _ = highs(Aeq, beq, c)
    # the reduced LP with the coordinate cost has the same optimum
    red, _ = highs(kron_A(m, n), oracle.bvec(mu1, mu2), oracle.cost(m, n, u, v))
    assert abs(red - opt) <= 1e-9 * max(opt, 1.0)
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=2000000, coord_row=u,
                                 coord_col=v)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - opt) <= 1e-6 * opt


def test_nonuniform_cost_entries(oracle):
    """Spot entries of c against the bin positions (index map of A.1)."""
    m, n = 3, 4
    u = np.array([0.0, 0.5, 2.25])
    v = np.array([-1.0, 0.0, 3.0, 3.5])
    c = oracle.cost(m, n, u, v)
    # x1 index (j m + k) m + i <-> f1_{i,k,j}: (u_k - u_i)^2
    assert c[(2 * m + 2) * m + 0] == (2.25 - 0.0) ** 2
    assert c[(3 * m + 0) * m + 1] == 0.25
    # x2 index m^2 n + (l n + j) m + k <-> f2_{k,j,l}: (v_j - v_l)^2
    assert c[m * m * n + (3 * n + 0) * m + 1] == (-1.0 - 3.5) ** 2
    assert c[m * m * n + (1 * n + 2) * m + 2] == 9.0


@pytest.mark.parametrize("n", [9, 14])
def test_nonuniform_one_dimensional(oracle, n):
    rng = np.random.default_rng(n)
    mu1, mu2 = rand_hist(rng, 1, n, 0.2), rand_hist(rng, 1, n, 0.2)
    v = coords(rng, n)
    exact = w2_1d_positions(mu1.ravel(), mu2.ravel(), v)
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=2000000,
                                 coord_row=np.array([7.5]), coord_col=v)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - exact) <= 1e-6 * exact


@pytest.mark.parametrize("m,n", [(6, 8), (10, 7)])
def test_nonuniform_separable(oracle, m, n):
    rng = np.random.default_rng(m * n + 1)
    a1, a2 = rng.uniform(0.1, 1, m), rng.uniform(0.1, 1, m)
    b1, b2 = rng.uniform(0.1, 1, n), rng.uniform(0.1, 1, n)
    a1, a2, b1, b2 = (t / t.sum() for t in (a1, a2, b1, b2))
    u, v = coords(rng, m), coords(rng, n)
    exact = w2_1d_positions(a1, a2, u) + w2_1d_positions(b1, b2, v)
    _, _, _, _, res = oracle.hot(np.outer(a1, b1), np.outer(a2, b2), tol=1e-10,
                                 max_iter=2000000, coord_row=u, coord_col=v)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - exact) <= 1e-6 * exact


def test_coordinate_scaling_and_uniform_default(oracle):
    rng = np.random.default_rng(5)
    m, n = 6, 5
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    u, v = coords(rng, m), coords(rng, n)
    r1 = oracle.hot(mu1, mu2, tol=1e-9, max_iter=2000000, coord_row=u, coord_col=v)[4]
    r2 = oracle.hot(mu1, mu2, tol=1e-9, max_iter=2000000, coord_row=3 * u, coord_col=3 * v)[4]
    assert abs(r2["primal_obj"] - 9 * r1["primal_obj"]) <= 1e-6 * 9 * r1["primal_obj"]
    # the uniform grid given explicitly is the default path, bit for bit
    a = oracle.hot(mu1, mu2, fixed_iters=25)
    b = oracle.hot(mu1, mu2, fixed_iters=25, coord_row=np.arange(m, dtype=float),
                   coord_col=np.arange(n, dtype=float))
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("m,n", [(3, 4), (4, 4)])
def test_prop1_nonuniform(oracle, m, n):
    """Prop. 1 with non-uniform bins: on LP-exact reduced flows, Algorithm 1
    yields a plan with the exact marginals whose full cost equals the reduced
    optimum, which equals the full LP optimum."""
    rng = np.random.default_rng(31 * m + n)
    mu1, mu2 = rand_hist(rng, m, n, 0.1), rand_hist(rng, m, n, 0.1)
    u, v = coords(rng, m), coords(rng, n)
    st, x, red = oracle.simplex(kron_A(m, n), oracle.bvec(mu1, mu2), oracle.cost(m, n, u, v))
    assert st == 0
    src, dst, mass = oracle.recover(m, n, x)
    row, col = oracle.marginals(m, n, src, dst, mass)
    assert np.abs(row - mu1.ravel()).sum() <= 1e-12
    assert np.abs(col - mu2.ravel()).sum() <= 1e-12
    si, sj = np.divmod(src, n)
    di, dj = np.divmod(dst, n)
    cost = float(((u[si] - u[di]) ** 2 + (v[sj] - v[dj]) ** 2) @ mass)
    full, _ = highs(*full_ot_lp_xy(mu1, mu2, u, v))
    assert abs(cost - red) <= 1e-10 * max(1.0, red)
    assert abs(full - red) <= 1e-9 * max(1.0, red)
