"""FP64 CPU oracle for HOT (arXiv 2408.00598) -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package.  It shares no code with the GPU library.
"""
