"""MI355X (gfx950) real-time TD-DFTB density-matrix propagation.

The compute path is the HIP library libtddftb.so (C ABI in
include/tddftb.h); ``paper_1912_03174_amd.tddftb`` is its ctypes binding.
"""
from . import tddftb  # noqa: F401
from .tddftb import Propagator, TdError  # noqa: F401
