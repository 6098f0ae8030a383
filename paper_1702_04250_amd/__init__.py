"""MI355X-native PPPM particle-mesh path (particle map, make_rho, Poisson,
fieldforce ik/ad, energy and its adjoint).  The compute lives in
``lib/libpppm_mi355x.so`` (HIP kernels for gfx950 behind the C ABI of
``include/pppm.h``); this package only marshals arguments."""
from .binding import (PPPMEnergy, PPPMError, Plan, compute_noalloc, declared_functions, last_error, load, make_params,
                      pppm_energy, validate)

__all__ = ["Plan", "PPPMEnergy", "PPPMError", "pppm_energy", "load", "validate", "make_params",
           "declared_functions", "last_error", "compute_noalloc"]
