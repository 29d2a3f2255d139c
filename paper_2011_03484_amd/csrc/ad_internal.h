// Launchers of the tangent / adjoint kernels (ad_kernels.hip).
#pragma once
#include "internal.h"

namespace tpm {

hipError_t launch_aos_to_soa(const double* r, const double* v, double* o, int64_t n,
                             hipStream_t st);
hipError_t launch_soa_to_aos(const double* o, double* r, double* v, int64_t n, hipStream_t st);

// Fields per particle and step of an adjoint tape: the state at the step's
// start (6), the acceleration of its opening kick (3), and the root of its
// drift's Kepler equation with its sin and cos - 1 (3).
constexpr int AD_TAPE_FIELDS = 12;

// Steps [s0, s1) of the map for n particles from state `in` ([6][n]) to `out`
// (may be null); writes every step the particle carries out to `tape`
// ([s1-s0][AD_TAPE_FIELDS][n], may be null).  mode 0: first segment, removal records
// initialised; 1: records read and updated; 2: recompute of a recorded run
// (particle i advances through steps s < dstep[i]; records untouched).
hipError_t launch_ad_segment(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, const double* in, double* out, double* tape,
                             int64_t* dstep, int32_t* reason, int32_t* planet, int mode,
                             hipStream_t st);

// Adjoint of steps [s0, s1) from the segment's tape; lam ([6][n]) in/out.
hipError_t launch_ad_reverse(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, const double* tape, double* lam,
                             const int64_t* dstep, hipStream_t st);

// Tangent of steps [s0, s1): state and tangent ([6][n] each) in/out.
hipError_t launch_ad_tangent(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, double* st_, double* tg, int32_t* reason,
                             bool first, hipStream_t st);

}  // namespace tpm
