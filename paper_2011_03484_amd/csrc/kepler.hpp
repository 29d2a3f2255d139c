// Kepler drift with the f and g functions (Zhang & Gladman 2021, sec. 2.2,
// drift step and the difference form of Kepler's equation), FP64, gfx950.
//
// With r0 = |r|, u = r.v and alpha = 2/r0 - v^2/mu = 1/a, the mean motion is
// n = sqrt(mu alpha) alpha, ec = 1 - r0 alpha = e cos E0 and
// es = u sqrt(alpha/mu) = e sin E0.  The change x of eccentric anomaly over a
// step dt solves F(x) = x - ec sin x + es (1 - cos x) - n dt = 0, and
//   f = 1 + (a/r0)(cos x - 1),      g = dt + (sin x - x)/n,
//   fdot = -a^2 n sin x / (r1 r0),  gdot = 1 + (a/r1)(cos x - 1),
// with r1 = a F'(x), give r' = f r + g v and v' = fdot r + gdot v.
//
// Particle version (drift_fixed): at most k Newton steps from a fixed
// starting guess (sec. 2.2: a fixed iteration count, since the slowest lane of
// a group sets the group's time).  A lane stops early only once its iterate
// has converged to rounding (kepler_newton), so the result is the k-step
// result up to an ulp or two, and the wavefront leaves the loop when every
// lane has stopped.  The starter is the
// second-order series root x0 = dM/(1-ec) - es dM^2 / (2 (1-ec)^3), clamped to
// dM +- 2(|ec|+|es|) (a bracket of the root).  The drift is refused (returns
// false) when the orbit is unbound or |F(x_k)| > ftol; mean anomaly steps
// beyond pi are reduced by whole periods.
#pragma once
#include "dmath.hpp"
#include "internal.h"

namespace tpm {

constexpr double TWO_PI_HI = 0x1.921fb54442d18p+2;
constexpr double TWO_PI_LO = 0x1.1a62633145c07p-52;
constexpr double INV_TWO_PI = 0x1.45f306dc9c883p-3;


// sin/cos of an iterate; SHORT when every argument of the solve is known to
// lie within +-0.78 (see short_args), so the pi/2 reduction is skipped (the
// values are those of the full path up to the polynomial's evaluation order);
// otherwise each call checks by itself.  Only the planet map takes the SHORT
// form, evaluated by Horner's rule (see sincos_poly_horner).
template <bool SHORT>
TPM_DEV void sincos_it(double x, double& s, double& c) {
  if (SHORT) sincos_poly_horner(x, s, c);
  else sincos(x, s, c);
}

// A lane's starter (clamped to dM +- w, w = 2(|ec| + |es|)), root and Newton
// iterates stay within 0.66 of zero when |dM| <= 0.45 and w <= 0.2: then
// e <= 0.1, the root lies within 2e of dM, F' >= 1 - e and |F''| <= e, so one
// Newton step from the starter (at most 0.4 from the root) lands within 0.01
// of the root and later steps closer still.
TPM_DEV bool short_args(double dM, double w) {
  return __builtin_fabs(dM) <= 0.45 && w <= 0.2;
}

// At most kiters Newton steps on F(x) = x - ec sin x + es (1 - cos x) - dM
// from xk.  A lane stops after the first step whose correction is at most
// 2^-30 |x|: the error left after that step is below
// e/(2(1-e)) (2^-30 |x|)^2, under one ulp of x for e <= 0.99 and |x| <= 4, so
// the rest of the fixed count could only move x by rounding.  The stop is each
// lane's own decision, so the result of a particle does not depend on which
// particles share its wavefront; the wavefront leaves the loop once all its
// lanes have stopped, after two steps at the least.  Lanes with a NaN state
// (unbound orbits) never stop early; lanes that start with done set take no
// part.
//
// Returns the root and, in (s, c), its sine and cosine.  A lane's (s, c) are
// fixed in the step where it stops, like its root: from sin/cos of the point
// x of that step and the step's correction d (the root is x - d,
// |d| <= 2^-30 |x - d|), the first-order rotation
//   sin(x - d) = s - c d,  cos(x - d) = c + s d
// leaves out terms of size d^2/2 <= 2^-61 (x - d)^2, under 0.05 ulp of
// either value.  Lanes still iterating when the step budget runs out get
// sin/cos of their last iterate afresh; lanes that start with done set get
// (0, 1) (their xk is 0).  Each lane's values depend only on its own
// iterates, whichever lanes share its wavefront.
template <bool SHORT>
TPM_DEV double kepler_newton(double ec, double es, double dM, int kiters, bool done, double xk,
                             double& s, double& c) {
  bool converged = false;   // wave-uniform: every lane stopped
  s = 0.0;
  c = 1.0;
  for (int it = 0; it < kiters; ++it) {
    if (it >= 2 && wave_all(done)) {
      converged = true;
      break;
    }
    double sv, cv;
    sincos_it<SHORT>(xk, sv, cv);
    double F = fma_(-ec, sv, fma_(es, 1.0 - cv, xk - dM));
    double Fp = fma_(-ec, cv, fma_(es, sv, 1.0));
    double xn = fma_(-F, rcp_newton(Fp), xk);
    const double d = xk - xn;
    bool small = __builtin_fabs(d) <= 0x1p-30 * __builtin_fabs(xn);
    const double sn = fma_(-cv, d, sv), cn = fma_(sv, d, cv);
    s = done ? s : sn;
    c = done ? c : cn;
    xk = done ? xk : xn;
    done = done | small;
  }
  if (!converged) {
    double sf, cf;
    sincos_it<SHORT>(xk, sf, cf);
    s = done ? s : sf;
    c = done ? c : cf;
  }
  return xk;
}

// Newton for the planet map: as kepler_newton, but no lane freezes.  The
// planet map's wavefront always holds the same bodies in the same lanes, so
// its results cannot depend on which lanes share it.  Every lane iterates
// until the last step of each non-idle lane was a correction of at most
// 2^-30 |x|, and its sin/cos come from that last step's rotation (as in
// kepler_newton); at most 40 steps, after which sin/cos are evaluated afresh.
// Idle lanes (dM = 0, x = 0) stay at x = 0.  Lanes beyond the bodies may
// carry NaN (their central-body term sits at zero distance), so idle lanes
// enter every wave-wide test through their idle flag.
template <bool SHORT>
TPM_DEV double planet_newton(double ec, double es, double dM, bool idle, double xk, double& s,
                             double& c) {
  bool done = idle;
  for (int it = 0; it < 40; ++it) {
    if (it >= 2 && wave_all(done)) return xk;
    double sv, cv;
    sincos_it<SHORT>(xk, sv, cv);
    const double F = fma_(-ec, sv, fma_(es, 1.0 - cv, xk - dM));
    const double Fp = fma_(-ec, cv, fma_(es, sv, 1.0));
    const double xn = fma_(-F, rcp_newton(Fp), xk);
    const double d = xk - xn;
    done = idle | (__builtin_fabs(d) <= 0x1p-30 * __builtin_fabs(xn));
    s = fma_(-cv, d, sv);
    c = fma_(sv, d, cv);
    xk = xn;
  }
  sincos_it<SHORT>(xk, s, c);
  return xk;
}

// The particles' Newton solve from the starter xk, with sin/cos of its result.
// (Each sin/cos decides its short path by itself: one copy of the loop keeps
// the particle kernel's registers within budget.)
TPM_DEV double kepler_solve(double ec, double es, double dM, int kiters, double xk, double& s,
                            double& c) {
  return kepler_newton<false>(ec, es, dM, kiters, false, xk, s, c);
}

// Drift (x, v) by dt about mass mu with k fixed Newton iterations.  Writes the
// drifted state into (x, v) on every lane; where the return value is false
// (the drift is refused) that state is meaningless and the caller keeps its
// own copy of the old one.
TPM_DEV bool drift_fixed(const KepConst& K, double dt, int kiters, double ftol,
                         double& x, double& y, double& z,
                         double& vx, double& vy, double& vz) {
  double r2 = fma_(x, x, fma_(y, y, z * z));
  double v2 = fma_(vx, vx, fma_(vy, vy, vz * vz));
  double u = fma_(x, vx, fma_(y, vy, z * vz));
  double r0, rinv;
  sqrt_rsqrt(r2, r0, rinv);
  double alpha = fma_(-v2, K.inv_mu, 2.0 * rinv);
  bool bound = alpha > 0.0;
  double sa, rsa;
  sqrt_rsqrt(alpha, sa, rsa);            // NaN for unbound lanes, never selected
  double a = rsa * rsa;                  // 1/alpha
  a = fma_(a, fma_(-alpha, a, 1.0), a);  // one correction to ~1 ulp
  double n = K.sqrt_mu * sa * alpha;
  double ninv = K.inv_sqrt_mu * rsa * a; // 1/n
  double ec = fma_(-r0, alpha, 1.0);
  double es = u * sa * K.inv_sqrt_mu;
  double dM = n * dt;
  // reduce dM to (-pi, pi]; keep dt itself when no whole period is removed
  double q = __builtin_rint(dM * INV_TWO_PI);
  double dMr = fma_(-q, TWO_PI_HI, dM);
  dMr = fma_(-q, TWO_PI_LO, dMr);
  double dte = (q == 0.0) ? dt : dMr * ninv;
  dM = dMr;
  // starter (only a first guess: a one-refinement reciprocal is enough)
  double om = 1.0 - ec;
  double oinv = rcp_newton(om);
  double t = dM * oinv;
  double xk = t * fma_(-0.5 * es * t, oinv, 1.0);
  double w = 2.0 * (__builtin_fabs(ec) + __builtin_fabs(es));
  xk = __builtin_fmin(__builtin_fmax(xk, dM - w), dM + w);
  double s, c;
  xk = kepler_solve(ec, es, dM, kiters, xk, s, c);
  double F = fma_(-ec, s, fma_(es, 1.0 - c, xk - dM));
  double Fp = fma_(-ec, c, fma_(es, s, 1.0));
  // one compare: an unbound orbit counts as an infinite residual
  const bool ok = (bound ? __builtin_fabs(F) : __builtin_inf()) <= ftol;
  double cm1 = c - 1.0;
  double r1 = a * Fp;
  double r1inv = rcp(r1);
  double f = fma_(a * rinv, cm1, 1.0);
  double g = fma_(s - xk, ninv, dte);
  double fd = -(a * a) * n * s * rinv * r1inv;
  double gd = fma_(a * r1inv, cm1, 1.0);
  double nx = fma_(f, x, g * vx), ny = fma_(f, y, g * vy), nz = fma_(f, z, g * vz);
  double nvx = fma_(fd, x, gd * vx), nvy = fma_(fd, y, gd * vy), nvz = fma_(fd, z, gd * vz);
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return ok;
}

// Converged drift for the planets (a handful of lanes in one wavefront):
// Newton until every lane has made a step whose correction is at most
// 2^-30 |x| (converged to rounding; planet_newton), at most 40 steps.  A lane
// that holds no body, or whose body is found unbound (the return value is then
// false), drifts for no time on a stand-in bound orbit (alpha = 1): dM = 0,
// x = 0, f = gdot = 1 and g = fdot = 0 exactly, so its state is left as it
// was without any select on the result.
TPM_DEV bool drift_converged(const KepConst& K, double dt, bool lane_on,
                             double& x, double& y, double& z,
                             double& vx, double& vy, double& vz) {
  double r2 = fma_(x, x, fma_(y, y, z * z));
  double v2 = fma_(vx, vx, fma_(vy, vy, vz * vz));
  double u = fma_(x, vx, fma_(y, vy, z * vz));
  double r0, rinv;
  sqrt_rsqrt(lane_on ? r2 : 1.0, r0, rinv);
  double alpha = fma_(-v2, K.inv_mu, 2.0 * rinv);
  const bool bound = alpha > 0.0;
  const bool idle = !(lane_on && bound);
  alpha = idle ? 1.0 : alpha;
  dt = idle ? 0.0 : dt;
  double sa, rsa;
  sqrt_rsqrt(alpha, sa, rsa);
  double a = rsa * rsa;
  a = fma_(a, fma_(-alpha, a, 1.0), a);
  double n = K.sqrt_mu * sa * alpha;
  double ninv = K.inv_sqrt_mu * rsa * a;
  double ec = fma_(-r0, alpha, 1.0);
  double es = u * sa * K.inv_sqrt_mu;
  double dM = n * dt;
  double q = __builtin_rint(dM * INV_TWO_PI);
  double dMr = fma_(-q, TWO_PI_HI, dM);
  dMr = fma_(-q, TWO_PI_LO, dMr);
  double dte = (q == 0.0) ? dt : dMr * ninv;
  dM = dMr;
  double om = 1.0 - ec;
  double oinv = rcp_newton(om);   // a first guess only: one refinement is enough
  double t = dM * oinv;
  double xk = t * fma_(-0.5 * es * t, oinv, 1.0);
  double w = 2.0 * (__builtin_fabs(ec) + __builtin_fabs(es));
  xk = __builtin_fmin(__builtin_fmax(xk, dM - w), dM + w);
  double s, c;
  if (wave_all(idle | short_args(dM, w))) xk = planet_newton<true>(ec, es, dM, idle, xk, s, c);
  else xk = planet_newton<false>(ec, es, dM, idle, xk, s, c);
  double Fp = fma_(-ec, c, fma_(es, s, 1.0));
  double cm1 = c - 1.0;
  double r1 = a * Fp;
  double r1inv = rcp(r1);
  double f = fma_(a * rinv, cm1, 1.0);
  double g = fma_(s - xk, ninv, dte);
  double fd = -(a * a) * n * s * rinv * r1inv;
  double gd = fma_(a * r1inv, cm1, 1.0);
  double nx = fma_(f, x, g * vx), ny = fma_(f, y, g * vy), nz = fma_(f, z, g * vz);
  double nvx = fma_(fd, x, gd * vx), nvy = fma_(fd, y, gd * vy), nvz = fma_(fd, z, gd * vz);
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return bound;
}

}  // namespace tpm
