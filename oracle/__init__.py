"""CPU FP64 oracle for real-time TD-DFTB propagation (test infrastructure).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it. The GPU library
never calls it, and it shares no code with the GPU library.
"""
from .tddftb import *  # noqa: F401,F403
