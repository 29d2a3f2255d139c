// Two-body drift in universal variables, for the orbits the elliptic
// fixed-iteration drift refuses: unbound ones, and bound ones whose Kepler
// solve has not converged after the fixed count (the near-parabolic case the
// paper's Kepler-solver paragraph in sec. 2.2 leaves to future work).  It is
// valid on every conic, so a particle on such an orbit goes on being
// integrated instead of being removed.  Only the lanes that need it run it
// (rare, lane-divergent by nature), so it is written for robustness, not for
// wavefront uniformity.
//
// Textbook formulation (universal anomaly chi, alpha = 2/r0 - v0^2/mu,
// sigma0 = r0.v0 / sqrt(mu), z = alpha chi^2, Stumpff functions
// C(z) = (1 - cos sqrt z)/z and S(z) = (sqrt z - sin sqrt z)/z^(3/2), with
// their hyperbolic continuations for z < 0):
//   T(chi) = r0 chi + sigma0 chi^2 C(z) + (1 - alpha r0) chi^3 S(z) = sqrt(mu) dt,
//   T'(chi) = r(chi) = chi^2 C(z) + sigma0 chi (1 - z S(z)) + r0 (1 - z C(z)) > 0,
// so T is increasing and the root is bracketed between 0 and any chi where
// T - sqrt(mu) dt changes sign.  The Lagrange coefficients are
//   f = 1 - chi^2 C / r0,   g = (r0 chi (1 - z S) + sigma0 chi^2 C)/sqrt(mu),
//   fdot = sqrt(mu) chi (z S - 1)/(r r0),   gdot = 1 - chi^2 C / r,
// with g written through the equation itself (dt - chi^3 S / sqrt(mu) would
// cancel near pericentre).
#pragma once
#include <hip/hip_runtime.h>

#include "dmath.hpp"

namespace tpm {

// C(z) and S(z).  For |z| <= 4 their power series
//   C = sum_k (-z)^k / (2k+2)!,  S = sum_k (-z)^k / (2k+3)!
// (terms through k = 13: the first one left out is below 4^14/29! < 1e-22 of
// a value >= 0.08); beyond, the closed forms, whose subtractions lose at most
// a factor 3 there (sqrt|z| >= 2).
TPM_DEV void stumpff_cs(double z, double& C, double& S) {
  if (__builtin_fabs(z) <= 4.0) {
    // Horner from the highest term: C = 1/2! (1 - z/(3*4) (1 - z/(5*6) (...)))
    double c = 1.0, s = 1.0;
#pragma unroll
    for (int k = 13; k >= 1; --k) {
      c = fma_(-z * (1.0 / ((2.0 * k + 1.0) * (2.0 * k + 2.0))), c, 1.0);
      s = fma_(-z * (1.0 / ((2.0 * k + 2.0) * (2.0 * k + 3.0))), s, 1.0);
    }
    C = 0.5 * c;
    S = s / 6.0;
  } else if (z > 0.0) {
    const double q = sqrt(z);
    C = (1.0 - cos(q)) / z;
    S = (q - sin(q)) / (z * q);
  } else {
    const double q = sqrt(-z);
    C = (cosh(q) - 1.0) / (-z);
    S = (sinh(q) - q) / (-z * q);
  }
}

// Drift (x, v) by dt about mu in universal variables.  Returns false (state
// unchanged) if no finite result is reached.
TPM_DEV bool drift_universal(double mu, double dt, double& x, double& y, double& z,
                             double& vx, double& vy, double& vz) {
  if (dt == 0.0) return true;
  const double r0 = sqrt(x * x + y * y + z * z);
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double smu = sqrt(mu);
  const double sig = (x * vx + y * vy + z * vz) / smu;
  const double alpha = 2.0 / r0 - v2 / mu;
  const double target = smu * dt;
  const double sgn = dt > 0.0 ? 1.0 : -1.0;
  // G(chi) = sgn (T(chi) - target): increasing in sgn * chi, G(0) < 0
  double C, S, rr;
  auto G = [&](double chi) {
    const double zz = alpha * chi * chi;
    stumpff_cs(zz, C, S);
    const double c2 = chi * chi;
    rr = c2 * C + sig * chi * (1.0 - zz * S) + r0 * (1.0 - zz * C);
    return sgn * (r0 * chi + sig * c2 * C + (1.0 - alpha * r0) * c2 * chi * S - target);
  };
  // bracket [0, hi] (in the direction of dt) by doubling from target / r0
  double lo = 0.0, hi = target / r0;
  int guard = 0;
  while (!(G(hi) >= 0.0)) {
    if (!__builtin_isfinite(hi) || ++guard > 1100) return false;
    lo = hi;
    hi *= 2.0;
  }
  // Newton from the bracket's midpoint, falling back to bisection whenever a
  // step leaves the bracket; stops at a step of at most 4 ulp of chi or a
  // bracket that narrow.
  double chi = 0.5 * (lo + hi);
  for (int it = 0; it < 300; ++it) {
    const double g = G(chi);
    if (g == 0.0) break;
    if (g < 0.0) lo = chi;
    else hi = chi;
    double nc = chi - sgn * g / rr;
    const bool inside = sgn > 0.0 ? (nc > lo && nc < hi) : (nc < lo && nc > hi);
    if (!inside) nc = 0.5 * (lo + hi);
    const double step = __builtin_fabs(nc - chi);
    chi = nc;
    const double tol = 0x1p-50 * __builtin_fabs(chi);
    if (step <= tol || __builtin_fabs(hi - lo) <= tol) break;
  }
  (void)G(chi);   // C, S and r at the root
  const double zz = alpha * chi * chi;
  const double c2 = chi * chi;
  const double f = 1.0 - c2 * C / r0;
  const double g = (r0 * chi * (1.0 - zz * S) + sig * c2 * C) / smu;
  const double fd = smu * chi * (zz * S - 1.0) / (rr * r0);
  const double gd = 1.0 - c2 * C / rr;
  if (!(__builtin_isfinite(f) && __builtin_isfinite(g) && __builtin_isfinite(fd) &&
        __builtin_isfinite(gd)))
    return false;
  const double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
  const double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy, nvz = fd * z + gd * vz;
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return true;
}

}  // namespace tpm
