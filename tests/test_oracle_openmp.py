"""The oracle's OpenMP build (the same source with its independent loops on
several threads, used only to time the oracle on several cores) gives results
bit-identical to the serial build."""
import numpy as np
import pytest

from oracle import oracle as O


def _pair(m, n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, (m, n)) * (rng.uniform(size=(m, n)) < 0.8)
    b = rng.uniform(0.0, 1.0, (m, n))
    a[0, 0] += 1e-3
    return a / a.sum(), b / b.sum()


@pytest.mark.parametrize("m,n", [(1, 5), (7, 4), (24, 24), (33, 17)])
def test_fixed_iterations_bit_identical(m, n):
    a, b = _pair(m, n, 10 * m + n)
    ser = O.hot(a, b, fixed_iters=25, restart=False)
    par = O.hot(a, b, fixed_iters=25, restart=False, threads=True)
    for u, v in zip(ser[:4], par[:4]):
        assert np.array_equal(u, v)
    assert ser[4] == par[4]


def test_converged_with_restarts_and_variants_bit_identical():
    a, b = _pair(12, 20, 7)
    for kw in ({}, {"sigma_update": True}, {"admm_rho": 1.7}):
        ser = O.hot(a, b, tol=1e-7, max_iter=100000, **kw)
        par = O.hot(a, b, tol=1e-7, max_iter=100000, threads=True, **kw)
        assert ser[4] == par[4]
        assert ser[4]["converged"] == 1
        for u, v in zip(ser[:4], par[:4]):
            assert np.array_equal(u, v)
