"""Autotuner: picks a launch shape, records it in a JSON-lines cache that a
fresh context can load, and tuned solves still meet the oracle tolerance."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu


def test_autotune_and_cache(tmp_path, oracle):
    need_gpu()
    from paper_2408_00598_amd import hot, workloads
    pairs = workloads.batch_pairs(6, sides=(16, 24, 32))
    dp = [(dev(a), dev(b)) for a, b in pairs]
    c = ctx()
    cache = str(tmp_path / "tune.jsonl")
    best = c.autotune(dp, iters=20, cache_path=cache, prec=hot.HOT_FP32_STREAM)
    assert best["item_elems"] >= 2048 and best["unroll"] in (1, 2)
    assert best["us_per_iter"] > 0 and best["default_us_per_iter"] > 0
    line = json.loads(open(cache).read().strip().splitlines()[-1])
    assert line["item_elems"] == best["item_elems"] and line["fp32"] == 1
    c2 = hot.Context(0)
    assert c2.autotune_load(cache)
    res = c2.batch_solve(dp, tol=1e-6, max_iter=200000, prec=hot.HOT_FP32_STREAM)
    for (a, b), r in zip(pairs, res):
        _, _, _, _, o = oracle.hot(a, b, tol=1e-6, max_iter=200000)
        assert r["status"] == 0
        assert abs(r["primal_obj"] - o["primal_obj"]) <= 1e-4 * abs(o["primal_obj"])
