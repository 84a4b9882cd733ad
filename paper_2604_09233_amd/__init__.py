"""MI355X (gfx950) non-Fourier SENSE: E, E^H, E^H E and CG as HIP kernels.

The compute lives in libnfs.so (C ABI in include/nfs.h); ``nfs`` is its thin
ctypes binding.
"""
from .nfs import (  # noqa: F401
    NfsError,
    Problem,
    apply_E,
    apply_EH,
    apply_EHE,
    cg_solve,
    context,
    lib,
)
