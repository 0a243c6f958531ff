"""CPU oracle for polynomial-matrix multiplication mod p (test infrastructure).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU library never does.
"""
from .oracle import *  # noqa: F401,F403
