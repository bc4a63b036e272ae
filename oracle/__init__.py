"""Plain FP64 CPU oracle for the batched MSG hot path (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It shares no code with the HIP path.
"""
