"""Compile the C oracle into oracle/_build/libhot_oracle.so (gcc, -O2).

Test infrastructure: the oracle is the CPU reference the GPU path is checked
against; building it is not using it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libhot_oracle.so")
LIB_OMP = os.path.join(OUT_DIR, "libhot_oracle_omp.so")  # same source, -fopenmp
SRC = os.path.join(HERE, "hot_oracle.c")


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"]


def build(openmp: bool = False, quiet: bool = True, sanitize_to: str = "") -> str:
    """The serial oracle, or (openmp) the same source with its independent
    loops on several threads, for multi-core timing only.  sanitize_to: build
    the serial oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    into this path instead (the sanitizer test loads it)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    out = sanitize_to or (LIB_OMP if openmp else LIB)
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", *(["-fopenmp"] if openmp else []),
           *(SANITIZE if sanitize_to else []), SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(out + ".tmp", out)
    return out


def ensure_built(openmp: bool = False) -> str:
    lib = LIB_OMP if openmp else LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        build(openmp=openmp)
    return lib


if __name__ == "__main__":
    print(build(quiet=False))
    print(build(openmp=True, quiet=False))
    sys.exit(0)
