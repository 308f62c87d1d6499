"""Plain FP64 CPU oracle (test infrastructure only; see ``oracle/lbm.py``).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the HIP product path."""
