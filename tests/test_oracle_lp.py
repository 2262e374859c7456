"""Pins of the oracle's optimisation results.

* The oracle's dense Bland simplex against an independent LP solver (HiGHS)
  on random LPs and on OT LPs.
* Reduced model = full OT model (the equivalence the paper takes from
  Auricchio et al., Sec. 2.1, and uses in the proof of Prop. 1).
* HOT (Algorithm 2) run to a tight tolerance reaches the exact LP optimum.
* Closed forms: 1 x n and n x 1 grids (1-D W2 by quantile coupling),
  translation (W2^2 = |shift|^2), separable products (sum of 1-D W2^2), and
  the marginal lower bound on any instance.
* Per-iteration identities from the appendix: A x_bar = b exactly, the
  nonnegative complementary x_tilde (def:tx, def:tx-prop), and the O(1/k)
  KKT bound of Prop. prop:complexity.
"""
import numpy as np
import pytest

from lp_helpers import full_ot_lp, highs, kron_A, rand_hist, reduced_lp


def test_simplex_matches_highs_random(oracle):
    rng = np.random.default_rng(11)
    for trial in range(20):
        rows, cols = int(rng.integers(2, 9)), int(rng.integers(9, 25))
        A = rng.integers(-3, 4, size=(rows, cols)).astype(float)
        x0 = rng.uniform(0, 1, cols) * (rng.uniform(size=cols) < 0.5)
        b = A @ x0                       # feasible by construction
        c = rng.uniform(0.1, 2.0, cols)  # bounded below on x >= 0
        st, x, obj = oracle.simplex(A, b, c)
        ref, _ = highs(A, b, c)
        assert st == 0
        assert abs(obj - ref) <= 1e-9 * max(1, abs(ref))
        assert np.abs(A @ x - b).max() <= 1e-9 and x.min() >= -1e-12


@pytest.mark.parametrize("m,n,zeros", [(2, 2, 0), (2, 3, 0), (3, 3, 0.3), (4, 4, 0), (3, 5, 0.2)])
def test_reduced_equals_full_lp(oracle, m, n, zeros):
    rng = np.random.default_rng(100 * m + n)
    mu1, mu2 = rand_hist(rng, m, n, zeros), rand_hist(rng, m, n, zeros)
    Af, bf, cf = full_ot_lp(mu1, mu2)
    Ar, br, cr = reduced_lp(mu1, mu2, oracle)
    st_f, _, full = oracle.simplex(Af, bf, cf)
    st_r, xr, red = oracle.simplex(Ar, br, cr)
    ref, _ = highs(Af, bf, cf)
    assert st_f == 0 and st_r == 0
    assert abs(full - ref) <= 1e-9 * max(1, ref)
    assert abs(red - full) <= 1e-9 * max(1, full)
    # reduced primal feasibility through the oracle's own A
    np.testing.assert_allclose(oracle.A(m, n, xr), br, atol=1e-12)


@pytest.mark.parametrize("m,n", [(2, 3), (3, 3), (4, 4), (5, 5), (6, 6), (3, 6)])
def test_hot_reaches_lp_optimum(oracle, m, n):
    rng = np.random.default_rng(5 * m + n)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    Ar, br, cr = reduced_lp(mu1, mu2, oracle)
    st, _, opt = oracle.simplex(Ar, br, cr)
    assert st == 0
    xb, yb, zb, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=400000)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - opt) <= 1e-6 * abs(opt)
    assert abs(res["dual_obj"] - opt) <= 1e-6 * abs(opt)


@pytest.mark.parametrize("shape", [(1, 9), (9, 1), (1, 16)])
def test_one_dimensional_closed_form(oracle, shape):
    m, n = shape
    rng = np.random.default_rng(m + 2 * n)
    mu1, mu2 = rand_hist(rng, m, n, 0.2), rand_hist(rng, m, n, 0.2)
    w2 = oracle.w2_1d(mu1.ravel(), mu2.ravel())
    # CDF closed form against an independent LP solve of the 1-D problem
    L = m * n
    Aeq, beq, c = full_ot_lp(mu1.reshape(1, L), mu2.reshape(1, L))
    ref, _ = highs(Aeq, beq, c)
    assert abs(w2 - ref) <= 1e-10
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=400000)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - w2) <= 1e-6 * max(w2, 1e-3)


def test_w2_1d_small_cases(oracle):
    # Dirac to Dirac: squared distance; mass split symmetric: exact value.
    a = np.array([1.0, 0, 0, 0]); b = np.array([0, 0, 0, 1.0])
    assert oracle.w2_1d(a, b) == 9.0
    a = np.array([0.5, 0, 0.5]); b = np.array([0, 1.0, 0])
    assert oracle.w2_1d(a, b) == 1.0


@pytest.mark.parametrize("n,shift", [(8, (2, 1)), (10, (0, 3)), (9, (-2, -2))])
def test_translation_closed_form(oracle, n, shift):
    rng = np.random.default_rng(n)
    a, b = shift
    mu1 = np.zeros((n, n))
    lo_i, lo_j = max(0, -a), max(0, -b)
    hi_i, hi_j = n - max(0, a), n - max(0, b)
    box = rng.uniform(0.2, 1.0, size=(hi_i - lo_i, hi_j - lo_j))
    box[rng.uniform(size=box.shape) < 0.3] = 0
    mu1[lo_i:hi_i, lo_j:hi_j] = box
    mu1 /= mu1.sum()
    mu2 = np.zeros_like(mu1)
    mu2[lo_i + a:hi_i + a, lo_j + b:hi_j + b] = mu1[lo_i:hi_i, lo_j:hi_j]
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=400000)
    exact = a * a + b * b
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - exact) <= 1e-6 * exact


@pytest.mark.parametrize("m,n", [(6, 8), (10, 10)])
def test_separable_closed_form(oracle, m, n):
    rng = np.random.default_rng(m * n)
    u1, u2 = rng.uniform(0.1, 1, m), rng.uniform(0.1, 1, m)
    v1, v2 = rng.uniform(0.1, 1, n), rng.uniform(0.1, 1, n)
    u1, u2, v1, v2 = (t / t.sum() for t in (u1, u2, v1, v2))
    mu1, mu2 = np.outer(u1, v1), np.outer(u2, v2)
    exact = oracle.w2_1d(u1, u2) + oracle.w2_1d(v1, v2)
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=400000)
    assert res["converged"] == 1
    assert abs(res["primal_obj"] - exact) <= 1e-6 * exact


def test_marginal_lower_bound(oracle):
    rng = np.random.default_rng(42)
    for _ in range(3):
        mu1, mu2 = rand_hist(rng, 7, 6), rand_hist(rng, 7, 6)
        lb = oracle.w2_1d(mu1.sum(1), mu2.sum(1)) + oracle.w2_1d(mu1.sum(0), mu2.sum(0))
        _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-9, max_iter=400000)
        assert res["primal_obj"] >= lb - 1e-6 * lb


def test_iteration_identities(oracle):
    """A x_bar = b at every k; x_tilde >= 0 and <x_tilde, z_bar> = 0."""
    m, n = 4, 5
    rng = np.random.default_rng(9)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    c = oracle.cost(m, n)
    b = oracle.bvec(mu1, mu2)
    for k in (1, 2, 7, 30):
        xb, yb, zb, s, res = oracle.hot(mu1, mu2, fixed_iters=k)
        assert np.linalg.norm(oracle.A(m, n, xb) - b) <= 1e-12 * (1 + np.linalg.norm(xb))
        sig = res["sigma"]
        xt = xb + sig * (oracle.AT(m, n, yb) + zb - c)
        assert xt.min() >= -1e-12 * np.abs(xt).max()
        assert abs(xt @ zb) <= 1e-12 * (np.linalg.norm(xt) * np.linalg.norm(zb) + 1e-300)
        assert zb.min() >= 0.0


def test_halpern_rate_bound(oracle):
    """||R(w_bar^k)|| <= (sigma+1)/sigma * R0/(k+1) with R0 = ||x* + sigma z*||
    (w^0 = 0), Prop. prop:complexity; (x*, z*) from a tight solve."""
    m, n = 3, 4
    rng = np.random.default_rng(21)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    c = oracle.cost(m, n)
    b = oracle.bvec(mu1, mu2)
    sigma = 0.05
    xs, ys, zs, _, res = oracle.hot(mu1, mu2, tol=1e-12, max_iter=2000000, sigma=sigma)
    assert res["converged"] == 1
    R0 = np.linalg.norm(xs + sigma * zs)
    for k in (0, 1, 5, 20, 100, 400):
        xb, yb, zb, _, _ = oracle.hot(mu1, mu2, fixed_iters=k, sigma=sigma, restart=False)
        r1 = b - oracle.A(m, n, xb)
        r2 = zb - np.maximum(zb - xb, 0.0)
        r3 = c - oracle.AT(m, n, yb) - zb
        nrm = np.sqrt(r1 @ r1 + r2 @ r2 + r3 @ r3)
        assert nrm <= 1.001 * (sigma + 1) / sigma * R0 / (k + 1)


@pytest.mark.parametrize("m,n", [(3, 4), (5, 5)])
def test_generalized_admm_reaches_lp_optimum(oracle, m, n):
    """The ADMM baseline (Step 4 replaced by the rho = 1.7 relaxation,
    Sec. 4.1) converges to the same LP optimum."""
    rng = np.random.default_rng(3 * m + n)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    Ar, br, cr = reduced_lp(mu1, mu2, oracle)
    st, _, opt = oracle.simplex(Ar, br, cr)
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=2000000, admm_rho=1.7)
    assert st == 0 and res["converged"] == 1 and res["restarts"] == 0
    assert abs(res["primal_obj"] - opt) <= 1e-6 * abs(opt)


def test_absolute_kkt_is_residual_map_norm(oracle):
    """||R(w_bar)|| of the complexity proposition, recomputed from the
    exported iterate with numpy, equals the reported absolute KKT, and the
    absolute stopping rule stops on it."""
    m, n = 4, 5
    rng = np.random.default_rng(12)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    c, b = oracle.cost(m, n), oracle.bvec(mu1, mu2)
    xb, yb, zb, _, res = oracle.hot(mu1, mu2, fixed_iters=37)
    r1 = b - oracle.A(m, n, xb)
    r2 = zb - np.maximum(zb - xb, 0.0)
    r3 = c - oracle.AT(m, n, yb) - zb
    ref = np.sqrt(r1 @ r1 + r2 @ r2 + r3 @ r3)
    assert abs(res["kkt_abs"] - ref) <= 1e-12 * ref
    _, _, _, _, r = oracle.hot(mu1, mu2, tol=1e-5, abs_kkt=True, max_iter=400000)
    assert r["converged"] == 1 and r["kkt_abs"] <= 1e-5


@pytest.mark.parametrize("m,n,seed", [(3, 4, 1), (5, 3, 3)])
def test_complexity_bound_along_trajectory(oracle, m, n, seed):
    """Prop. complexity: for Algorithm 2 without restarts and w^0 = 0,
    ||R(w_bar^k)|| <= ((sigma+1)/sigma) R0/(k+1) with
    R0 = ||x* + sigma z*|| for a KKT point (x*, y*, z*).  The KKT point comes
    from HiGHS (primal x*, equality duals y*, z* = c - A^T y*), not from the
    oracle."""
    from scipy.optimize import linprog
    rng = np.random.default_rng(seed)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    A, b, c = reduced_lp(mu1, mu2, oracle)
    r = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    xs, ys = r.x, r.eqlin.marginals
    zs = c - A.T @ ys
    assert zs.min() > -1e-9 and abs(c @ xs - b @ ys) < 1e-9
    sigma = np.linalg.norm(b) / np.linalg.norm(c)
    R0 = np.linalg.norm(xs + sigma * zs)
    for K in (1, 2, 5, 17, 60, 250):
        res = oracle.hot(mu1, mu2, fixed_iters=K, restart=False)[4]
        assert res["sigma"] == pytest.approx(sigma, rel=1e-14)
        assert res["kkt_abs"] <= (sigma + 1) / sigma * R0 / (K + 1) * (1 + 1e-9), K


@pytest.mark.parametrize("m,n", [(3, 4), (5, 5), (4, 6)])
def test_sigma_update_reaches_lp_optimum(oracle, m, n):
    """Optional sigma re-balancing at restarts (sigma <- ||dx|| / ||A^T dy||
    over the last epoch) still converges to the HiGHS optimum."""
    rng = np.random.default_rng(7 * m + n)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    Ar, br, cr = reduced_lp(mu1, mu2, oracle)
    opt, _ = highs(Ar, br, cr)
    _, _, _, _, res = oracle.hot(mu1, mu2, tol=1e-10, max_iter=400000, sigma_update=True)
    assert res["converged"] == 1 and res["restarts"] >= 1
    assert abs(res["primal_obj"] - opt) <= 1e-6 * abs(opt)


def test_sigma_update_is_scale_consistent(oracle):
    """sigma carries mass/cost units: scaling every cost by t (grid positions
    by sqrt(t)) must scale every sigma by 1/t and leave the iteration count
    unchanged; the reciprocal rule (||A^T dy|| / ||dx||) would not."""
    m, n = 6, 7
    rng = np.random.default_rng(11)
    mu1, mu2 = rand_hist(rng, m, n), rand_hist(rng, m, n)
    u, v = np.arange(m, dtype=float), np.arange(n, dtype=float)
    t = 16.0  # sqrt(t) = 4: positions scale exactly
    a = oracle.hot(mu1, mu2, tol=1e-6, max_iter=400000, sigma_update=True,
                   coord_row=u, coord_col=v)[4]
    b = oracle.hot(mu1, mu2, tol=1e-6, max_iter=400000, sigma_update=True,
                   coord_row=4 * u, coord_col=4 * v)[4]
    assert a["converged"] == 1 and b["converged"] == 1 and a["restarts"] >= 2
    assert a["iters"] == b["iters"] and a["restarts"] == b["restarts"]
    assert abs(b["sigma"] * t - a["sigma"]) <= 1e-9 * a["sigma"]
    assert abs(b["primal_obj"] - t * a["primal_obj"]) <= 1e-9 * t * a["primal_obj"]


def test_sigma_update_off_is_default(oracle):
    rng = np.random.default_rng(3)
    mu1, mu2 = rand_hist(rng, 5, 6), rand_hist(rng, 5, 6)
    a = oracle.hot(mu1, mu2, tol=1e-6)
    b = oracle.hot(mu1, mu2, tol=1e-6, sigma_update=False)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4] == b[4]
