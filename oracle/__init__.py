"""FP64 CPU oracle for the reduced QMC matrix-vector product.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The HIP product path never imports it.
"""
