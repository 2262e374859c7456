"""Degenerate grids: 1 x 1 (zero cost everywhere, sigma falls back to 1)."""
import numpy as np


def test_one_by_one_grid(oracle):
    mu = np.ones((1, 1))
    xb, yb, zb, s, res = oracle.hot(mu, mu, tol=1e-12, max_iter=1000)
    assert res["sigma"] == 1.0
    assert res["converged"] == 1
    assert abs(res["primal_obj"]) <= 1e-12
    # the only flows: f1 = f2 = mu
    np.testing.assert_allclose(xb, [1.0, 1.0], atol=1e-9)
