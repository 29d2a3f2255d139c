// Interface of the sampled-diagnostics and snapshot kernels (diag_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tpm {

// Device pointers and constants of one sample boundary.  Accumulators and
// snapshot entries are indexed by slot (the caller's particle index).
struct DiagArgs {
  // accumulators (null: no diagnostics, snapshot only)
  double* emax;         // [n] largest sampled eccentricity, -1 before any sample
  int64_t* estep;       // [n] first sampled step reaching it, -1 before any sample
  int32_t* flags;       // [n][nres] bit 0: phi within 10 deg of 0; bit 1: of 180 deg
  double* lo;           // [n][nres] range of phi - pi, folded into (-pi, pi]
  double* hi;
  int nres;
  int p[2], q[2];
  int ref;              // internal index of the reference planet
  double mu0;           // central mass (particles' elements)
  double mu_ref;        // mu0 + mu of the reference planet (its elements)
  const double* vref;   // device: heliocentric velocity of the reference planet at the boundary
  // snapshot (null: none): r, v [n][3], step [n], reason [n], elements [n][6]
  double* snap_r;
  double* snap_v;
  int64_t* snap_step;
  int32_t* snap_reason;
  double* snap_el;
};

// Sample the active particles of the working set at global step `step`, whose
// planet-table row is `row`.
hipError_t launch_sample(const SysConst& S, Work w, const int32_t* d_nactive, int n_upper,
                         const double* row, int64_t step, const DiagArgs& D, hipStream_t st);
// Snapshot entries of every slot from the removal records (before launch_sample).
hipError_t launch_snapshot_base(Out out, int n, double mu0, const DiagArgs& D, hipStream_t st);
// Accumulators of n particles to their starting values.
hipError_t launch_diag_reset(int n, const DiagArgs& D, hipStream_t st);

}  // namespace tpm
