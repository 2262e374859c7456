"""Failure paths through the C ABI, each forced from the host so that every
kernel still exits normally:
* HOT_E_NUMERIC: a context created with HOT_TEST_NAN_AFTER writes a NaN (a
  value, not a fault) into the flow state between two graph launches; the
  next check must stop the solve with HOT_E_NUMERIC.
* HOT_E_CANCELLED: hot_server_cancel ends queued and resident problems with
  HOT_E_CANCELLED, and the server keeps serving afterwards.
"""
import time

import numpy as np
import pytest

from gpu_helpers import dev, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_nan_in_state_gives_numeric(monkeypatch, prec):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    mu1, mu2 = workloads.pair_small(3)
    monkeypatch.setenv("HOT_TEST_NAN_AFTER", "2")
    c = hot.Context(0)
    monkeypatch.delenv("HOT_TEST_NAN_AFTER")
    res, _ = c.solve(dev(mu1), dev(mu2), tol=1e-10, max_iter=100000, prec=prec,
                     raise_on_error=False)
    assert res["return_status"] == hot.HOT_E_NUMERIC and res["status"] == hot.HOT_E_NUMERIC
    # stopped at the first check after the poisoned graph
    assert 2 * 20 <= res["iters"] <= 4 * 20
    # the same problem on a context without the hook is fine
    ok, _ = hot.Context(0).solve(dev(mu1), dev(mu2), tol=1e-6, prec=prec)
    assert ok["status"] == 0


@pytest.mark.parametrize("shared", [False, True])
def test_server_cancel(shared):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    c = hot.Context(0)
    srv = hot.Server(c, max_slots=2, shared=shared)
    keep = []
    for t in range(6):  # two resident, four queued; none can finish soon
        a, b = (dev(x) for x in workloads.pair_medium("blobs", pair=t, n=64))
        keep.append((a, b))
        srv.submit(a, b, t, tol=1e-13, max_iter=2_000_000)
    t0 = time.time()
    while srv.stats()["resident"] < 2 and time.time() - t0 < 30:
        time.sleep(0.01)
    time.sleep(0.05)
    srv.cancel()
    assert srv.drain(60.0) == hot.HOT_OK
    res = srv.poll(16)
    assert sorted(r["tag"] for r in res) == list(range(6))
    assert all(r["status"] == hot.HOT_E_CANCELLED for r in res)
    resident = [r for r in res if r["iters"] > 0]
    assert len(resident) == 2 and all(np.isfinite(r["primal_obj"]) for r in resident)
    # still serving
    a, b = (dev(x) for x in workloads.pair_small(1))
    srv.submit(a, b, 99, tol=1e-5)
    assert srv.drain(60.0) == hot.HOT_OK
    (r,) = srv.poll(4)
    assert r["tag"] == 99 and r["status"] == 0
    srv.close()
