"""CPU FP64 reference of explicit DUGKS and IDUGKS (arXiv:1709.01819).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark.  The product path never imports it.
"""
from .oracle import Oracle, build, load, quadrature_1d  # noqa: F401
