"""Seeded synthetic inputs for the non-Fourier SENSE hot path.

This package only draws and shapes input arrays (coordinates, basis values,
spiral trajectories, field terms, B0 maps, coil sensitivities, phantoms and
unit noise).  It holds none of the method's arithmetic: it never evaluates the
encoding operator, its adjoint or the solver.  Both the FP64 oracle (tests)
and the GPU library (tests, benchmark) take their inputs from here.
"""
from .inputs import (  # noqa: F401
    CONFIGS,
    solid_harmonics,
    grid_coords,
    make_config,
    random_problem,
    dft_problem,
    unit_noise,
    batched_slices,
    prescan,
    reconstruction_mask,
    restrict_voxels,
)
