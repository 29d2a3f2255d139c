// Planet-table rows from a history of planet states instead of the planet map
// (sec. 2.2: the planet positions the particles share may come from any
// source, such as interpolation from a history file).
//
// Records k = 0..nrec-1 at increasing times t_k hold heliocentric planet
// positions and velocities.  Row n of a run is the time t0 + n dt; between the
// records around it each planet follows the cubic Hermite interpolant, the
// cubic that matches both records' positions and velocities.  Written in
// powers of s = (t - t_a)/h, h = t_b - t_a:
//   r(s)  = r_a + s (h v_a + s (c2 + s c3)),
//   c2 = 3 (r_b - r_a) - h (2 v_a + v_b),   c3 = 2 (r_a - r_b) + h (v_a + v_b),
//   dr/dt = (h v_a + s (2 c2 + 3 s c3)) / h.
// The row's indirect term is h0 = -sum_j mu_j r_j / |r_j|^3 of the
// interpolated positions.  Unlike the planet map this has no chain in time:
// one thread per row.
#include <hip/hip_runtime.h>

#include "history_internal.h"
#include "internal.h"

namespace tpm {

// Index k of the record interval [t_k, t_k+1] holding time x (t_0 <= x <=
// t_{nrec-1}; the largest k <= nrec - 2 with t_k <= x).
__device__ __forceinline__ int64_t find_interval(const double* __restrict__ t, int64_t nrec,
                                                 double x) {
  int64_t lo = 0, hi = nrec - 2;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (t[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One planet's interpolated position (and velocity) at s in the interval
// starting at record k.
__device__ __forceinline__ void hermite(const HistDev& H, int64_t k, int j, double s, double h,
                                        double* r, double* v) {
  const int64_t k1 = H.nrec > 1 ? k + 1 : k;
  const double* ra = H.r + (k * H.np + j) * 3;
  const double* rb = H.r + (k1 * H.np + j) * 3;
  const double* va = H.v + (k * H.np + j) * 3;
  const double* vb = H.v + (k1 * H.np + j) * 3;
  for (int c = 0; c < 3; ++c) {
    if (h > 0.0) {
      const double hva = h * va[c];
      const double c2 = 3.0 * (rb[c] - ra[c]) - h * (2.0 * va[c] + vb[c]);
      const double c3 = 2.0 * (ra[c] - rb[c]) + h * (va[c] + vb[c]);
      r[c] = ra[c] + s * (hva + s * (c2 + s * c3));
      if (v) v[c] = (hva + s * (2.0 * c2 + 3.0 * s * c3)) / h;
    } else {
      r[c] = ra[c];
      if (v) v[c] = va[c];
    }
  }
}

// Rows [0, nrows) of a chunk whose row 0 is global step step0; vside (may be
// null) receives the planet velocities at rows 0 and nrows - 1, [2][np][3].
__global__ void __launch_bounds__(256)
history_rows(HistDev H, double* __restrict__ rows, int nrows, int64_t step0, double dt,
             double* __restrict__ vside) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const double x = H.t0 + (double)(step0 + i) * dt;
  const int64_t k = find_interval(H.t, H.nrec, x);
  const double h = H.nrec > 1 ? H.t[k + 1] - H.t[k] : 0.0;
  const double s = h > 0.0 ? (x - H.t[k]) / h : 0.0;
  const int rl = 3 * H.np + 3;
  double* row = rows + (size_t)i * rl;
  double h0[3] = {0.0, 0.0, 0.0};
  const bool edge = vside && (i == 0 || i == nrows - 1);
  for (int j = 0; j < H.np; ++j) {
    double r[3], v[3];
    hermite(H, k, j, s, h, r, edge ? v : nullptr);
    row[3 * j + 0] = r[0]; row[3 * j + 1] = r[1]; row[3 * j + 2] = r[2];
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double w = H.mu[j] / (r2 * sqrt(r2));
    h0[0] -= w * r[0]; h0[1] -= w * r[1]; h0[2] -= w * r[2];
    if (edge) {
      double* o = vside + (i == 0 ? 0 : 3 * H.np) + 3 * j;
      o[0] = v[0]; o[1] = v[1]; o[2] = v[2];
      if (nrows == 1) {
        double* o2 = vside + 3 * H.np + 3 * j;
        o2[0] = v[0]; o2[1] = v[1]; o2[2] = v[2];
      }
    }
  }
  row[3 * H.np + 0] = h0[0]; row[3 * H.np + 1] = h0[1]; row[3 * H.np + 2] = h0[2];
}

hipError_t launch_history_rows(const HistDev& H, double* rows, int nrows, int64_t step0, double dt,
                               double* vside, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(history_rows, dim3((nrows + 255) / 256), dim3(256), 0, st, H, rows, nrows,
                     step0, dt, vside);
  return hipGetLastError();
}

}  // namespace tpm
