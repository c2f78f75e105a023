"""FP64 CPU oracle for replica-averaged Brownian dynamics.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark. The product package never imports it.
"""
