// Sampled diagnostics and snapshots of the particles (the paper's applications,
// secs. 3.3, 4.1 and 4.2, and its periodic output of the particle arrays,
// sec. 2.2).  These kernels run at sample boundaries only (every `every`
// steps, at the end of a particle launch), never inside the step loop.
//
//  * sample_kernel   - per active particle of the working set: osculating
//    heliocentric elements; the largest eccentricity and the first sampled
//    step that reached it (sec. 3.3); for up to two resonances p:q with a
//    reference planet the resonant angle
//        phi = p lambda - q lambda_ref - (p - q) varpi        (sec. 4.1)
//    folded into (-pi, pi] about 0 and about pi, with flag bit 0 set by a
//    sample within 10 degrees of 0 and bit 1 by one within 10 degrees of pi
//    (the libration criterion of sec. 4.2: a librator about pi never comes
//    within 10 degrees of 0), and the range of phi - pi; optionally the
//    particle's state and elements into a snapshot buffer.
//  * snapshot_base   - snapshot entries of removed particles (their removal
//    records), written before sample_kernel fills in the active ones.
#include <hip/hip_runtime.h>

#include "diag_internal.h"
#include "internal.h"
#include "particle.hpp"

namespace tpm {

// Osculating heliocentric elements (a, e, inc, node, peri, M) of (r, v) about
// mu by the two-body relations: a from the vis-viva energy; e as the length of
// the eccentricity vector ((v^2 - mu/r) r - (r.v) v)/mu; inc and node from the
// angular momentum h = r x v; e cos E = 1 - r/a and e sin E = r.v/sqrt(mu a)
// give the eccentric anomaly E, the mean anomaly M = E - e sin E and the true
// anomaly f (tan f = sqrt(1 - e^2) sin E / (cos E - e), both arguments scaled
// by e so that a circular orbit gives f = E = 0); the argument of latitude u is
// the angle of r from the ascending node in the orbit plane, and the argument
// of pericentre is u - f.  The mean longitude node + peri + M is then well
// defined on a circular orbit.  Unbound orbits get M = f = NaN.
TPM_DEV void osc_elements(double mu, double x, double y, double z, double vx, double vy,
                          double vz, double* el) {
  const double r = sqrt(x * x + y * y + z * z);
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double rv = x * vx + y * vy + z * vz;
  const double a = 1.0 / (2.0 / r - v2 / mu);
  const double hx = y * vz - z * vy, hy = z * vx - x * vz, hz = x * vy - y * vx;
  const double hxy = sqrt(hx * hx + hy * hy);
  const double h = sqrt(hxy * hxy + hz * hz);
  const double kk = v2 - mu / r;
  const double ex = (kk * x - rv * vx) / mu, ey = (kk * y - rv * vy) / mu,
               ez = (kk * z - rv * vz) / mu;
  const double e = sqrt(ex * ex + ey * ey + ez * ez);
  const double inc = atan2(hxy, hz);
  const double node = atan2(hx, -hy);
  const double cn = cos(node), sn = sin(node);
  // m = (h / |h|) x (cos node, sin node, 0): 90 degrees ahead of the node line
  const double mx = -hz * sn / h, my = hz * cn / h, mz = (hx * sn - hy * cn) / h;
  const double u = atan2(x * mx + y * my + z * mz, x * cn + y * sn);
  const double ec = 1.0 - r / a;
  const double es = rv / sqrt(mu * a);
  const double E = atan2(es, ec);
  const double f = atan2(sqrt(1.0 - e * e) * es, ec - e * e);
  el[0] = a;
  el[1] = e;
  el[2] = inc;
  el[3] = node;
  el[4] = u - f;
  el[5] = E - es;
}

constexpr double TEN_DEG = M_PI / 18.0;
constexpr double TWO_PI_D = 2.0 * M_PI;

template <int NP>
__global__ void __launch_bounds__(256)
sample_kernel(Work w, const int32_t* __restrict__ d_nactive, const double* __restrict__ row,
              PlanetConst<NP> P, double rmax2, int64_t step, DiagArgs D) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_nactive || w.status[i] != ST_ACTIVE) return;
  const int k = w.slot[i];
  const double x = w.x[i], y = w.y[i], z = w.z[i];
  const double vx = w.vx[i], vy = w.vy[i], vz = w.vz[i];
  // the boundary's removal test (the particle kernel applies the same one at
  // this step): a particle removed here is not sampled
  double ax, ay, az;
  const int hit = accel<NP>(row, P, x, y, z, ax, ay, az);
  const bool escaped = fma_(x, x, fma_(y, y, z * z)) > rmax2;
  double el[6];
  osc_elements(D.mu0, x, y, z, vx, vy, vz, el);
  if (D.snap_r) {
    D.snap_r[3 * k + 0] = x; D.snap_r[3 * k + 1] = y; D.snap_r[3 * k + 2] = z;
    D.snap_v[3 * k + 0] = vx; D.snap_v[3 * k + 1] = vy; D.snap_v[3 * k + 2] = vz;
    D.snap_step[k] = (hit >= 0 || escaped) ? step : -1;
    D.snap_reason[k] = hit >= 0 ? ST_ENCOUNTER : escaped ? ST_ESCAPE : ST_ACTIVE;
    for (int c = 0; c < 6; ++c) D.snap_el[6 * k + c] = el[c];
  }
  if (!D.emax || hit >= 0 || escaped) return;
  if (el[1] > D.emax[k]) {
    D.emax[k] = el[1];
    D.estep[k] = step;
  }
  if (D.nres == 0) return;
  // the reference planet's mean longitude, from its position (table row) and
  // velocity (planet map) about mu0 + mu_ref
  double pel[6];
  const double* pr = row + 3 * D.ref;
  osc_elements(D.mu_ref, pr[0], pr[1], pr[2], D.vref[0], D.vref[1], D.vref[2], pel);
  const double lam_ref = pel[3] + pel[4] + pel[5];
  const double varpi = el[3] + el[4];
  const double lam = varpi + el[5];
  for (int q = 0; q < D.nres; ++q) {
    const double phi = D.p[q] * lam - D.q[q] * lam_ref - (D.p[q] - D.q[q]) * varpi;
    const double w0 = remainder(phi, TWO_PI_D);
    const double w180 = remainder(phi - M_PI, TWO_PI_D);
    int32_t f = D.flags[D.nres * k + q];
    if (__builtin_fabs(w0) < TEN_DEG) f |= 1;
    if (__builtin_fabs(w180) < TEN_DEG) f |= 2;
    D.flags[D.nres * k + q] = f;
    D.lo[D.nres * k + q] = fmin(D.lo[D.nres * k + q], w180);
    D.hi[D.nres * k + q] = fmax(D.hi[D.nres * k + q], w180);
  }
}

template <int NP>
static hipError_t sample_np(const SysConst& S, Work w, const int32_t* d_nactive, int n_upper,
                            const double* row, int64_t step, const DiagArgs& D, hipStream_t st) {
  PlanetConst<NP> P;
  for (int j = 0; j < NP; ++j) { P.mu[j] = S.mu[j]; P.rcrit2[j] = S.rcrit2[j]; }
  if (NP == 0) { P.mu[0] = 0.0; P.rcrit2[0] = 0.0; }
  hipLaunchKernelGGL(sample_kernel<NP>, dim3((n_upper + 255) / 256), dim3(256), 0, st, w, d_nactive,
                     row, P, S.rmax2, step, D);
  return hipGetLastError();
}

hipError_t launch_sample(const SysConst& S, Work w, const int32_t* d_nactive, int n_upper,
                         const double* row, int64_t step, const DiagArgs& D, hipStream_t st) {
  if (n_upper <= 0) return hipSuccess;
  switch (S.np) {
    case 0: return sample_np<0>(S, w, d_nactive, n_upper, row, step, D, st);
    case 1: return sample_np<1>(S, w, d_nactive, n_upper, row, step, D, st);
    case 2: return sample_np<2>(S, w, d_nactive, n_upper, row, step, D, st);
    case 3: return sample_np<3>(S, w, d_nactive, n_upper, row, step, D, st);
    case 4: return sample_np<4>(S, w, d_nactive, n_upper, row, step, D, st);
    case 5: return sample_np<5>(S, w, d_nactive, n_upper, row, step, D, st);
    case 6: return sample_np<6>(S, w, d_nactive, n_upper, row, step, D, st);
    case 7: return sample_np<7>(S, w, d_nactive, n_upper, row, step, D, st);
    case 8: return sample_np<8>(S, w, d_nactive, n_upper, row, step, D, st);
    default: return hipErrorInvalidValue;
  }
}

// Snapshot entries from the removal records (every slot; the active ones are
// overwritten by sample_kernel of the same boundary).
__global__ void __launch_bounds__(256)
snapshot_base(Out out, int n, double mu0, DiagArgs D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double x = out.r[3 * k + 0], y = out.r[3 * k + 1], z = out.r[3 * k + 2];
  const double vx = out.v[3 * k + 0], vy = out.v[3 * k + 1], vz = out.v[3 * k + 2];
  D.snap_r[3 * k + 0] = x; D.snap_r[3 * k + 1] = y; D.snap_r[3 * k + 2] = z;
  D.snap_v[3 * k + 0] = vx; D.snap_v[3 * k + 1] = vy; D.snap_v[3 * k + 2] = vz;
  D.snap_step[k] = out.step[k];
  D.snap_reason[k] = out.reason[k];
  double el[6];
  osc_elements(mu0, x, y, z, vx, vy, vz, el);
  for (int c = 0; c < 6; ++c) D.snap_el[6 * k + c] = el[c];
}

hipError_t launch_snapshot_base(Out out, int n, double mu0, const DiagArgs& D, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(snapshot_base, dim3((n + 255) / 256), dim3(256), 0, st, out, n, mu0, D);
  return hipGetLastError();
}

// Accumulators to their starting values: emax -1, estep -1, flags 0, lo +inf,
// hi -inf.
__global__ void __launch_bounds__(256) diag_reset(int n, DiagArgs D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  D.emax[k] = -1.0;
  D.estep[k] = -1;
  for (int q = 0; q < D.nres; ++q) {
    D.flags[D.nres * k + q] = 0;
    D.lo[D.nres * k + q] = __builtin_inf();
    D.hi[D.nres * k + q] = -__builtin_inf();
  }
}

hipError_t launch_diag_reset(int n, const DiagArgs& D, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_reset, dim3((n + 255) / 256), dim3(256), 0, st, n, D);
  return hipGetLastError();
}

}  // namespace tpm
