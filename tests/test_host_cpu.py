"""Host-side logic that runs without a GPU: the benchmark's argument and
cache handling, its traffic gate, and the seeded input generators."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_describe_names_precision_and_tolerance():
    b = _bench()
    from paper_2408_00598_amd import hot
    assert b.describe("w", hot.HOT_FP32_STREAM, 1e-4, False) == \
        "w, FP32 streams + FP64 reductions, rel KKT 1e-4"
    assert b.describe("w", hot.HOT_FP64, 1e-6, True) == \
        "w, FP64, rel KKT 1e-6, sigma re-balanced at restarts"


def test_cached_choice_matches_size_and_pair_classes(tmp_path):
    b = _bench()
    path = tmp_path / "cache.jsonl"
    rows = [
        {"arch": "gfx950", "fp32": 1, "size_class": 28, "pairs_class": 8, "item_elems": 4096},
        "not json",
        {"arch": "gfx950", "fp32": 1, "size_class": 28, "pairs_class": 8, "item_elems": 8192},
        {"arch": "gfx950", "fp32": 1, "size_class": 28, "pairs_class": 0, "item_elems": 65536},
        {"arch": "gfx950", "fp32": 0, "size_class": 28, "pairs_class": 8, "item_elems": 2048},
    ]
    path.write_text("\n".join(r if isinstance(r, str) else json.dumps(r) for r in rows) + "\n")
    total = 2 ** 28 + 5  # floor(log2) = 28
    hit = b.cached_choice(str(path), 1, total, 256)  # floor(log2(256)) = 8; the last line wins
    assert hit["item_elems"] == 8192
    assert b.cached_choice(str(path), 1, total, 1)["item_elems"] == 65536
    assert b.cached_choice(str(path), 0, total, 300)["item_elems"] == 2048
    assert b.cached_choice(str(path), 1, 2 ** 20, 256) is None
    assert b.cached_choice(str(tmp_path / "missing.jsonl"), 1, total, 256) is None


def test_traffic_is_reported_only_for_the_profiled_source_and_launch(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "paper_2408_00598_amd" / "csrc"
    src.mkdir(parents=True)
    for f in b.SLAB_SOURCES:
        (src / f).write_text(f"// {f} v1\n")
    sha = b.slab_source_sha256(str(tmp_path))
    h = hashlib.sha256()  # the digest is over name and contents of each file in turn
    for f in b.SLAB_SOURCES:
        h.update(f.encode() + b"\0" + (src / f).read_bytes())
    assert sha == h.hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "slab_pass_batched256_fp32_traffic.md").write_text(
        "# summary\n\nworkload: batched\nlaunch_config: item_elems=8192,unroll=2,vec_per_lane=2\n"
        f"traffic_bytes_per_launch: 2970000000\nkernel_source_sha256: {sha}\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    launch = "item_elems=8192,unroll=2,vec_per_lane=2"
    assert b.measured_traffic("batched", launch) == pytest.approx(2.97)
    assert b.measured_traffic("batched", "item_elems=4096,unroll=2,vec_per_lane=2") is None
    assert b.measured_traffic("pair128", launch) is None  # no summary for that workload
    (src / "hot_internal.h").write_text("// hot_internal.h v2\n")  # a struct it reads changed
    assert b.measured_traffic("batched", launch) is None
    (src / "hot_internal.h").write_text("// hot_internal.h v1\n")
    assert b.measured_traffic("batched", launch) == pytest.approx(2.97)
    (src / "hot_slab.hip").write_text("// kernel source v2\n")  # the kernel changed
    assert b.measured_traffic("batched", launch) is None


def test_seeds_and_histograms():
    from paper_2408_00598_amd import workloads as W
    assert W.seed_for(3, 7) == 240800598 + 3007
    pairs = W.batch_pairs(20)
    assert {a.shape[0] for a, _ in pairs} <= set(W.BATCH_SIDES)
    for a, b in pairs:
        assert a.shape == b.shape and a.shape[0] == a.shape[1]
        assert a.min() >= 0 and b.min() >= 0
        assert abs(a.sum() - 1) < 1e-12 and abs(b.sum() - 1) < 1e-12
    again = W.batch_pairs(20)
    assert all(np.array_equal(a, c) and np.array_equal(b, d)
               for (a, b), (c, d) in zip(pairs, again))


def test_serving_trace_shape():
    from paper_2408_00598_amd import workloads as W
    tr = W.serving_trace(rate=200.0, duration=30.0)
    t = np.array([r[0] for r in tr])
    assert np.all(np.diff(t) > 0) and t[-1] < 30.0
    assert abs(len(tr) / 30.0 - 200.0) < 200.0 * 0.05  # Poisson count, 5%
    assert {r[1] for r in tr} == set(W.SERVE_SIDES)
    frac = np.mean([r[2] == 1e-4 for r in tr])
    assert abs(frac - 0.7) < 0.03 and {r[2] for r in tr} == {1e-4, 1e-6}
    a, b = W.serving_pair(64, tr[0][3])
    assert a.shape == (64, 64) and abs(a.sum() - 1) < 1e-12 and abs(b.sum() - 1) < 1e-12
