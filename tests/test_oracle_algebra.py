"""Pins of the oracle's linear algebra against the paper's definitions.

* or_A / or_AT against A built from the Kronecker products of def:A1A2A3 and
  def:A4 (Sec. 2.1) -- catches any index, sign or ordering slip.
* A A^T against the blocks E1..E5 of eq. Mat:OT_AAT.
* Full row rank 3M-1 (the claim after def:A4).
* Prop. 3 (prop:linsol_OT) against a dense LAPACK solve of A A^T y = R.
"""
import numpy as np
import pytest

from lp_helpers import aat_blocks, kron_A

SHAPES = [(1, 1), (1, 5), (5, 1), (2, 3), (3, 2), (4, 4), (5, 7), (7, 5)]


def dense_from(op, m, n, length):
    cols = []
    for e in range(length):
        v = np.zeros(length)
        v[e] = 1.0
        cols.append(op(m, n, v))
    return np.array(cols).T


@pytest.mark.parametrize("m,n", SHAPES)
def test_A_matches_kronecker_definition(oracle, m, n):
    N, M3 = oracle.dims(m, n)
    assert N == m * m * n + m * n * n and M3 == 3 * m * n - 1
    Ak = kron_A(m, n)
    Ao = dense_from(oracle.A, m, n, N)
    assert Ao.shape == Ak.shape
    np.testing.assert_array_equal(Ao, Ak)


@pytest.mark.parametrize("m,n", SHAPES)
def test_AT_is_transpose(oracle, m, n):
    N, M3 = oracle.dims(m, n)
    Ak = kron_A(m, n)
    ATo = dense_from(oracle.AT, m, n, M3)
    np.testing.assert_array_equal(ATo, Ak.T)


@pytest.mark.parametrize("m,n", [(1, 4), (4, 1), (2, 3), (3, 3), (4, 6)])
def test_AAT_blocks_and_rank(oracle, m, n):
    Ak = kron_A(m, n)
    np.testing.assert_array_equal(Ak @ Ak.T, aat_blocks(m, n))
    assert np.linalg.matrix_rank(Ak) == 3 * m * n - 1


@pytest.mark.parametrize("m,n", SHAPES + [(6, 6), (3, 9)])
def test_prop3_solve_matches_dense_solve(oracle, m, n):
    rng = np.random.default_rng(7 + m * 31 + n)
    Ak = kron_A(m, n)
    R = rng.standard_normal(3 * m * n - 1) * 10.0 ** rng.uniform(-3, 3)
    y_dense = np.linalg.solve(Ak @ Ak.T, R)
    y = oracle.solve_aat(m, n, R)
    assert np.abs(y - y_dense).max() <= 1e-11 * max(1.0, np.abs(y_dense).max())
    # residual through the oracle's own operators
    r = oracle.A(m, n, oracle.AT(m, n, y)) - R
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(R) * (m + n)


def test_cost_and_b_vectors(oracle):
    m, n = 3, 4
    rng = np.random.default_rng(3)
    mu1 = rng.uniform(size=(m, n)); mu1 /= mu1.sum()
    mu2 = rng.uniform(size=(m, n)); mu2 /= mu2.sum()
    c = oracle.cost(m, n)
    # c^T x for x = indicator of f1_{i,k,j} / f2_{k,j,l}: eq. partite-graph objective
    x = np.zeros_like(c)
    x[(2 * m + 0) * m + 2] = 1.0   # f1_{i=2,k=0,j=2}: cost (0-2)^2
    assert c @ x == 4.0
    x[:] = 0
    x[m * m * n + (3 * n + 1) * m + 2] = 1.0  # f2_{k=2,j=1,l=3}: cost (1-3)^2
    assert c @ x == 4.0
    b = oracle.bvec(mu1, mu2)
    M = m * n
    assert np.all(b[:M] == 0)
    np.testing.assert_array_equal(b[M:2 * M], mu1.T.ravel())
    np.testing.assert_array_equal(b[2 * M:], mu2.T.ravel()[:-1])
