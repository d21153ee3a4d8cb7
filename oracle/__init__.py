"""FP64 CPU oracle of the coupled freezing step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path never routes through it.
"""
