"""Non-uniform bins on the GPU path, through the C ABI, against the oracle.

Bin (i,j) sits at (u_i, v_j); the slab passes read the positions from LDS
and the reduce/solve side uses the per-family cost tables.
* fixed trajectories equal the oracle's after k updates, elementwise;
* converged solves stop at the oracle's iteration with its objective;
* the uniform grid given explicitly is bit-identical to the default;
* a batch mixing uniform and non-uniform problems equals solo solves;
* the recovered plan has the non-uniform cost of the reduced objective.
"""
import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def close(a, b, tol, floor):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max()) <= tol * max(float(np.abs(b).max()), floor)


def case(m, n, seed, sort=True):
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(seed)
    mu1, mu2 = workloads.gaussian_blobs(m, n, 3, rng), workloads.gaussian_blobs(m, n, 3, rng)
    u, v = workloads.grid_lines(m, rng), workloads.grid_lines(n, rng)
    if not sort:
        u, v = rng.permutation(u), rng.permutation(v)
    return mu1, mu2, u + 2.5, v - 1.0


@pytest.mark.parametrize("m,n,sort", [(1, 9, True), (2, 3, True), (7, 5, False), (32, 32, True),
                                      (17, 40, False), (65, 33, True)])
@pytest.mark.parametrize("k", [1, 10, 100])
def test_nonuniform_fixed_trajectory(oracle, m, n, sort, k):
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2, u, v = case(m, n, 13 * m + n + k, sort)
    c = ctx()
    res, sol = c.solve(dev(mu1), dev(mu2), keep=True, max_iter=k, coord_row=dev(u),
                       coord_col=dev(v), flags=hot.HOT_FLAG_FIXED_ITERS)
    xb, yb, zb, s = (t.cpu().numpy() for t in sol.export())
    oxb, oyb, ozb, os_, ores = oracle.hot(mu1, mu2, fixed_iters=k, restart=False,
                                          coord_row=u, coord_col=v)
    assert res["iters"] == k
    # ||c|| is summed in another order on each side (FP64, ~N terms)
    assert abs(res["sigma"] - ores["sigma"]) <= 1e-12 * ores["sigma"]
    assert close(s, os_, 1e-10, 1e-3)
    assert close(yb, oyb, 1e-10, 1.0)
    assert close(xb, oxb, 1e-9, 1e-3)
    assert close(zb, ozb, 1e-9, 1.0)
    assert abs(res["primal_obj"] - ores["primal_obj"]) <= 1e-9 * abs(ores["primal_obj"]) + 1e-13


@pytest.mark.parametrize("m,n,tol", [(8, 8, 1e-6), (24, 16, 1e-5), (32, 32, 1e-4)])
def test_nonuniform_converged(oracle, m, n, tol):
    need_gpu()
    mu1, mu2, u, v = case(m, n, 7 * m + n)
    c = ctx()
    res, _ = c.solve(dev(mu1), dev(mu2), tol=tol, max_iter=200000, coord_row=dev(u),
                     coord_col=dev(v))
    _, _, _, _, o = oracle.hot(mu1, mu2, tol=tol, max_iter=200000, coord_row=u, coord_col=v)
    assert res["status"] == 0 and o["converged"] == 1
    assert res["iters"] == o["iters"] and res["restarts"] == o["restarts"]
    assert abs(res["primal_obj"] - o["primal_obj"]) <= 1e-6 * abs(o["primal_obj"])


def test_nonuniform_fp32_streams(oracle):
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2, u, v = case(16, 12, 99)
    c = ctx()
    res, _ = c.solve(dev(mu1), dev(mu2), tol=1e-6, max_iter=200000, coord_row=dev(u),
                     coord_col=dev(v), prec=hot.HOT_FP32_STREAM)
    _, _, _, _, o = oracle.hot(mu1, mu2, tol=1e-6, max_iter=200000, coord_row=u, coord_col=v)
    assert res["status"] == 0
    assert abs(res["primal_obj"] - o["primal_obj"]) <= 1e-4 * abs(o["primal_obj"])


def test_explicit_uniform_grid_is_default_bitwise():
    need_gpu()
    from paper_2408_00598_amd import hot
    mu1, mu2, _, _ = case(20, 28, 5)
    c = ctx()
    u, v = np.arange(20, dtype=float), np.arange(28, dtype=float)
    for prec in (hot.HOT_FP64, hot.HOT_FP32_STREAM):
        a, sa = c.solve(dev(mu1), dev(mu2), tol=1e-6, max_iter=200000, prec=prec, keep=True)
        b, sb = c.solve(dev(mu1), dev(mu2), tol=1e-6, max_iter=200000, prec=prec, keep=True,
                        coord_row=dev(u), coord_col=dev(v))
        for key in ("primal_obj", "dual_obj", "kkt", "iters", "restarts", "sigma"):
            assert a[key] == b[key], key
        for ta, tb in zip(sa.export(), sb.export()):
            assert bool((ta == tb).all())


def test_batch_mixing_uniform_and_nonuniform():
    need_gpu()
    c = ctx()
    cases = [case(12, 12, 1), case(16, 8, 2), case(9, 14, 3), case(12, 12, 4)]
    pairs = []
    for idx, (mu1, mu2, u, v) in enumerate(cases):
        extra = {} if idx % 2 else {"coord_row": dev(u), "coord_col": dev(v)}
        pairs.append((dev(mu1), dev(mu2), extra))
    batch = c.batch_solve(pairs, tol=1e-6, max_iter=200000)
    for (a, b, extra), rb in zip(pairs, batch):
        ra, _ = c.solve(a, b, tol=1e-6, max_iter=200000, **extra)
        assert ra["status"] == 0 and rb["status"] == 0
        assert ra["iters"] == rb["iters"] and ra["restarts"] == rb["restarts"]
        assert abs(ra["primal_obj"] - rb["primal_obj"]) <= 1e-12 * abs(ra["primal_obj"])


def test_nonuniform_plan_cost(oracle):
    need_gpu()
    m, n = 16, 12
    mu1, mu2, u, v = case(m, n, 21)
    c = ctx()
    res, sol = c.solve(dev(mu1), dev(mu2), tol=1e-7, max_iter=400000, keep=True,
                       coord_row=dev(u), coord_col=dev(v))
    src, dst, mass, err = sol.recover_plan()
    src, dst, mass = (t.cpu().numpy() for t in (src, dst, mass))
    assert err[2] <= 1e-12 and err[3] <= 1e-12
    si, sj = np.divmod(src, n)
    di, dj = np.divmod(dst, n)
    cost = float(((u[si] - u[di]) ** 2 + (v[sj] - v[dj]) ** 2) @ mass)
    o = oracle.hot(mu1, mu2, tol=1e-7, max_iter=400000, coord_row=u, coord_col=v)[4]
    assert abs(cost - o["primal_obj"]) <= 1e-5 * o["primal_obj"]


def test_nonfinite_positions_rejected():
    need_gpu()
    from paper_2408_00598_amd import hot
    c = ctx()
    mu = np.full((4, 4), 1 / 16)
    bad = np.array([0.0, 1.0, np.inf, 3.0])
    r, _ = c.solve(dev(mu), dev(mu), coord_row=dev(bad), raise_on_error=False)
    assert r["return_status"] == hot.HOT_E_INVALID and "finite" in c.last_error()
    r, _ = c.solve(dev(mu), dev(mu), coord_col=dev(np.array([0, 1, np.nan, 2.0])),
                   raise_on_error=False)
    assert r["return_status"] == hot.HOT_E_INVALID
