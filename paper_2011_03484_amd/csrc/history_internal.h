// Interface of the planet-history interpolation kernel (history.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpm {

// A planet history on the device: records k = 0..nrec-1 at times t[k]
// (increasing), heliocentric r, v [nrec][np][3] in the planets' integration
// order; row n of a run lies at time t0 + n dt.
struct HistDev {
  int np;
  int64_t nrec;
  const double* t;
  const double* r;
  const double* v;
  double mu[8];
  double t0;
};

// Rows [0, nrows) of a chunk starting at global step step0 (rows of 3 np + 3
// doubles: positions, then h0); vside (may be null) receives the velocities at
// the first and last rows, [2][np][3].
hipError_t launch_history_rows(const HistDev& H, double* rows, int nrows, int64_t step0, double dt,
                               double* vside, hipStream_t st);

}  // namespace tpm
