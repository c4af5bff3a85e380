"""CPU oracle (test infrastructure only): plain FP64 reference for the HIP path.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path never does.
"""
