"""CPU FP64 oracle for spin-adapted two-site DMRG (test infrastructure).

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the GPU library.
"""
