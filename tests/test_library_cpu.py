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


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a struct of include/hot.h, from gcc."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hot.h"', 'int main(void) {',
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("name", ["Problem", "Result", "ServerConfig"])
def test_binding_structs_match_header(tmp_path, name):
    """The ctypes structures of the binding have the header's size and field
    offsets (compiled with gcc against include/hot.h)."""
    from paper_2408_00598_amd import hot
    cls = getattr(hot, name)
    cname = {"Problem": "hot_problem", "Result": "hot_result",
             "ServerConfig": "hot_server_config"}[name]
    fields = [f for f, _ in cls._fields_]
    got = _c_layout(tmp_path, cname, fields)
    assert got[0] == C_sizeof(cls), (cname, got[0])
    for f, off in zip(fields, got[1:]):
        assert getattr(cls, f).offset == off, (cname, f)


def C_sizeof(cls):
    import ctypes
    return ctypes.sizeof(cls)


def test_binding_flag_constants_match_header():
    from paper_2408_00598_amd import hot
    text = open(os.path.join(ROOT, "include", "hot.h")).read()
    defs = dict(re.findall(r"#define (HOT_FLAG_[A-Z_]+) (0x[0-9a-f]+)u", text))
    assert set(defs) == {"HOT_FLAG_RESTART", "HOT_FLAG_FIXED_ITERS", "HOT_FLAG_ADMM",
                         "HOT_FLAG_ABS_KKT", "HOT_FLAG_SIGMA_UPDATE", "HOT_FLAG_ESCALATE"}
    for k, v in defs.items():
        assert getattr(hot, k) == int(v, 16), k
    srv = re.search(r"#define HOT_SERVER_SHARED (0x[0-9a-f]+)u", text)
    assert srv and hot.HOT_SERVER_SHARED == int(srv.group(1), 16)


@pytest.mark.parametrize("name,cname", [("Params", "or_params"), ("Result", "or_result")])
def test_oracle_binding_structs_match_header(tmp_path, name, cname):
    """Same check for the oracle's ctypes wrapper against oracle/hot_oracle.h."""
    import subprocess
    from oracle import oracle as O
    cls = getattr(O, name)
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "ol.c"
    body = [f'  printf("%zu\\n", sizeof({cname}));']
    body += [f'  printf("%zu\\n", offsetof({cname}, {f}));' for f in fields]
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hot_oracle.h"\n'
                   'int main(void) {\n' + "\n".join(body) + '\n  return 0;\n}\n')
    exe = tmp_path / "ol"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "oracle"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got[0] == C_sizeof(cls)
    for f, off in zip(fields, got[1:]):
        assert getattr(cls, f).offset == off, (cname, f)
