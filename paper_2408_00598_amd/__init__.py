"""HOT on MI355X: Halpern-accelerated optimal transport (arXiv 2408.00598).

The solver lives in ``lib/libhot.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/hot.h``); ``hot`` is its Python binding and ``workloads`` the
seeded synthetic input generators.
"""
from . import workloads  # noqa: F401
