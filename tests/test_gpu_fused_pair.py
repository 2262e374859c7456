"""Reduce and solve in one launch (HOT_FUSE_PAIR=1, k_pair_fused): the same
device code as the two-kernel iteration with a device-scope handshake
between the reduce and the solve workgroups of each pair, so every result
and every exported state must be bit-identical to the two-kernel run."""
import numpy as np
import pytest

from gpu_helpers import dev, need_gpu

pytestmark = pytest.mark.gpu

KEYS = ("primal_obj", "dual_obj", "kkt", "kkt_abs", "feaserr", "iters", "restarts", "status")


def contexts(monkeypatch):
    from paper_2408_00598_amd import hot
    monkeypatch.setenv("HOT_FUSE_PAIR", "0")
    split = hot.Context(0)
    monkeypatch.setenv("HOT_FUSE_PAIR", "1")
    fused = hot.Context(0)
    return split, fused


def pair(m, n, seed, kind="blobs"):
    from paper_2408_00598_amd import workloads
    rng = np.random.default_rng(workloads.seed_for(5, seed))
    if kind == "noise":
        return workloads.white_noise(m, n, rng), workloads.white_noise(m, n, rng)
    return workloads.gaussian_blobs(m, n, 3, rng), workloads.gaussian_blobs(m, n, 3, rng)


@pytest.mark.parametrize("m,n,prec_name,tol,flags_name", [
    (32, 32, "HOT_FP64", 1e-6, "HOT_FLAG_RESTART"),
    (128, 128, "HOT_FP32_STREAM", 1e-4, "HOT_FLAG_RESTART"),
    (70, 65, "HOT_FP64", 1e-6, "HOT_FLAG_SIGMA_UPDATE"),
    (20, 130, "HOT_FP32_STREAM", 1e-5, "HOT_FLAG_RESTART"),
])
def test_fused_single_pair_bitwise(monkeypatch, m, n, prec_name, tol, flags_name):
    need_gpu()
    from paper_2408_00598_amd import hot
    split, fused = contexts(monkeypatch)
    mu1, mu2 = pair(m, n, m * 1000 + n)
    a, b = dev(mu1), dev(mu2)
    flags = hot.HOT_FLAG_RESTART | getattr(hot, flags_name)
    kw = dict(tol=tol, max_iter=200000, prec=getattr(hot, prec_name), flags=flags)
    print(f"fused pair {m}x{n} {prec_name} tol={tol} {flags_name}", flush=True)
    r0, s0 = split.solve(a, b, keep=True, **kw)
    r1, s1 = fused.solve(a, b, keep=True, **kw)
    assert r0["status"] == hot.HOT_OK
    for k in KEYS:
        assert r1[k] == r0[k], (k, r1[k], r0[k])
    for x0, x1 in zip(s0.export(), s1.export()):
        assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())
    s0.free()
    s1.free()


def test_fused_batch_bitwise(monkeypatch):
    need_gpu()
    from paper_2408_00598_amd import hot
    split, fused = contexts(monkeypatch)
    shapes = [(32, 32), (48, 48), (64, 64), (96, 96), (128, 128), (40, 72), (17, 40), (65, 33)]
    pairs = [tuple(dev(x) for x in pair(m, n, 77 + q, "noise" if q % 2 else "blobs"))
             for q, (m, n) in enumerate(shapes)]
    for prec in (hot.HOT_FP32_STREAM, hot.HOT_FP64):
        kw = dict(tol=1e-4, max_iter=100000, prec=prec)
        print(f"fused batch prec={prec}", flush=True)
        r0 = split.batch_solve(pairs, **kw)
        r1 = fused.batch_solve(pairs, **kw)
        for q in range(len(pairs)):
            assert r0[q]["status"] == hot.HOT_OK
            for k in KEYS:
                assert r1[q][k] == r0[q][k], (q, k)
