"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle: the same C source built with -fsanitize=address,undefined, and
  the oracle's pin tests run against that build in a child interpreter (the
  ASan runtime preloaded), so an out-of-bounds access or undefined behaviour
  anywhere in the oracle aborts them.
* The library's host-side layout code (csrc/hot_layout.hip, plain C++) built
  with g++ and the same sanitizers into tests/sanitize/layout_check.cpp, which
  checks the layout's invariants over many shapes, batches and tunings.
The GPU kernels are not built with sanitizers (that needs a GPU ASan
runtime); only host code is.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_00598_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def test_layout_host_code_sanitized(tmp_path):
    _runtime("libasan.so")
    exe = tmp_path / "layout_check"
    subprocess.run(["g++", "-std=c++17", "-O1", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-I", CSRC, "-x", "c++",
                    os.path.join(CSRC, "hot_layout.hip"), "-x", "c++",
                    os.path.join(ROOT, "tests", "sanitize", "layout_check.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    from oracle import build as ob
    lib = ob.build(sanitize_to=str(tmp_path / "libhot_oracle_san.so"))
    env = dict(os.environ, HOT_ORACLE_LIB=lib, LD_PRELOAD=asan, PYTHONMALLOC="malloc",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *tests], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out
    assert " passed" in out
