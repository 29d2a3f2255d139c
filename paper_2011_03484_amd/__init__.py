"""FP64 test-particle mixed-variable symplectic integrator for AMD MI355X.

The compute path is the HIP library ``libtpmvs.so`` (C ABI in include/tpmvs.h);
this package is its ctypes binding plus seeded input generators
(:mod:`paper_2011_03484_amd.workloads`).  There is no CPU fallback: without the
built library every entry point raises.
"""
from ._lib import (ACTIVE, ENCOUNTER, ESCAPE, KEPLER, TPM_EDEVICE, TPM_EINVAL, TPM_ENOMEM, TPM_EPLANET,
                   TPM_ESTATE, TPM_OK, PlanetEncounterError, Simulation, TpmError, batch_integrate,
                   debug_drift, debug_drift_universal, debug_rsqrt, debug_sincos, hill_radius,
                   integrate_static, load, run_workload)

__all__ = ["ACTIVE", "ENCOUNTER", "ESCAPE", "KEPLER", "TPM_EDEVICE", "TPM_EINVAL", "TPM_ENOMEM",
           "TPM_EPLANET", "TPM_ESTATE", "TPM_OK", "PlanetEncounterError", "Simulation", "TpmError",
           "batch_integrate", "debug_drift", "debug_drift_universal", "debug_rsqrt", "debug_sincos",
           "hill_radius", "integrate_static", "load", "run_workload"]
