"""FP64 test-particle mixed-variable symplectic integrator for AMD MI355X.

The compute path is the HIP library ``libtpmvs.so`` (C ABI in include/tpmvs.h);
this package is its ctypes binding plus seeded input generators
(:mod:`paper_2011_03484_amd.workloads`).  There is no CPU fallback: without the
built library every entry point raises.
"""
from ._lib import (ACTIVE, ENCOUNTER, ESCAPE, KEPLER, PlanetEncounterError, Simulation, TpmError,
                   batch_integrate, debug_drift, debug_rsqrt, debug_sincos, hill_radius,
                   integrate_static, load, run_workload)

__all__ = ["ACTIVE", "ENCOUNTER", "ESCAPE", "KEPLER", "PlanetEncounterError", "Simulation",
           "TpmError", "batch_integrate", "debug_drift", "debug_rsqrt", "debug_sincos", "hill_radius",
           "integrate_static", "load", "run_workload"]
