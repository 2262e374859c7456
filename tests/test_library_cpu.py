"""Host-side checks of libhot that need no GPU: the library loads, exports
every symbol include/hot.h declares, and its pure host arithmetic
(footprint, plan capacity, status strings) is right.  No compute call."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hot.h")).read()
    return sorted(set(re.findall(r"\b(hot_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    from paper_2408_00598_amd import hot
    L = hot.lib()
    names = declared_symbols()
    assert "hot_solve" in names and "hot_recover_plan" in names and "hot_batch_submit" in names
    for name in names:
        assert hasattr(L, name), name


def test_plan_capacity_and_footprint():
    from paper_2408_00598_amd import hot
    for m, n in [(1, 1), (3, 5), (32, 32), (512, 512)]:
        M = m * n
        assert hot.plan_capacity(m, n) == M * (m + n - 1) + 2 * M - 1
    assert hot.plan_capacity(0, 4) == 0
    # footprint: three state buffers dominate; FP32 about half of FP64
    f64 = hot.footprint_bytes(512, 512, hot.HOT_FP64)
    f32 = hot.footprint_bytes(512, 512, hot.HOT_FP32_STREAM)
    N = 2 * 512 ** 3
    assert 3 * 8 * N <= f64 <= 3.3 * 8 * N
    assert 3 * 4 * N <= f32 <= 3.6 * 4 * N
    assert hot.footprint_bytes(0, 5, hot.HOT_FP64) == 0
    assert hot.footprint_bytes(2000, 5, hot.HOT_FP64) == 0
    assert hot.footprint_bytes(4, 4, 7) == 0


def test_status_strings():
    from paper_2408_00598_amd import hot
    assert hot.status_string(hot.HOT_OK) == "ok"
    assert "converged" in hot.status_string(hot.HOT_E_NOT_CONVERGED)


def test_no_gpu_context_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2408_00598_amd import hot
    with pytest.raises(hot.HotError):
        hot.Context(0)
