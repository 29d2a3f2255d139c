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
// lane has stopped.  The starter is the third-order series root of F = 0 in
// t = dM/(1-ec) (kepler_starter), clamped to dM +- 2(|ec|+|es|) (a bracket of
// the root).  The drift is refused (returns false) when the orbit is unbound
// or |F(x_k)| > ftol; mean anomaly steps beyond pi are reduced by whole
// periods.
#pragma once
#include "dmath.hpp"
#include "internal.h"

namespace tpm {

constexpr double TWO_PI_HI = 0x1.921fb54442d18p+2;
constexpr double TWO_PI_LO = 0x1.1a62633145c07p-52;
constexpr double INV_TWO_PI = 0x1.45f306dc9c883p-3;


// sin and cos - 1 of an iterate; SHORT when every argument of the solve is
// known to lie within +-0.78 (see short_args), so the pi/2 reduction is
// skipped (the values are those of the full path up to the polynomial's
// evaluation order); otherwise each call checks by itself.  Only the planet
// map takes the SHORT form, evaluated by Horner's rule (see
// sincos_poly_horner).  The solve and the f and g functions use cos x - 1
// (m below) rather than cos x: F = x - ec sin x - es m - dM,
// F' = (1 - ec) - ec m + es sin x, f = 1 + (a/r0) m, gdot = 1 + (a/r1) m, all
// free of the cancellation 1 - cos x would bring for small x.
template <bool SHORT>
TPM_DEV void sincos_it(double x, double& s, double& m) {
  if (SHORT) sincos_poly_horner(x, s, m);
  else sincosm1(x, s, m);
}

// A lane's starter (clamped to dM +- w, w = 2(|ec| + |es|)), root and Newton
// iterates stay within 0.66 of zero when |dM| <= 0.45 and w <= 0.2: then
// e <= 0.1, the root lies within 2e of dM, F' >= 1 - e and |F''| <= e, so one
// Newton step from the starter (at most 0.4 from the root) lands within 0.01
// of the root and later steps closer still.
TPM_DEV bool short_args(double dM, double w) {
  return __builtin_fabs(dM) <= 0.45 && w <= 0.2;
}

// Newton steps on F(x) = x - ec sin x + es (1 - cos x) - dM from xk.  With
// e <= |ec| + |es| = eb, |F''| <= e and 1 - e <= F' <= 1 + e, so a step
// x -> x - d, whose d = F(x)/F'(x) is at least (1-e)/(1+e) times the error of
// x, leaves an error of at most Q d^2 with
//   Q = eb (1 + eb)^2 / (2 (1 - eb)^3)      (kepler_bound; +inf for eb > 0.75).
// A lane stops after the first step with Q d^2 <= 2^-54 |x - d| and
// |d| <= 2^-28 (a quarter ulp at most is left), or with |d| <= 2^-30 |x - d|
// (the error then is below e/(2(1-e)) (2^-30 |x|)^2, under one ulp for
// e <= 0.99, |x| <= 4).  The stop is each lane's own decision, so the result of
// a particle does not depend on which particles share its wavefront; the
// wavefront leaves the loop once all its lanes have stopped.  Lanes with a
// NaN state (unbound orbits) never stop; lanes that start with done set take
// no part.
//
// The method's fixed count kiters decides failure: Fk receives F(x_k) of a
// lane still iterating after kiters steps (0 for a lane that stopped before;
// the drift is refused where |Fk| > ftol).  Such a lane's state is taken from
// up to KEPLER_EXTRA further steps: a lane that passes the failure rule has
// |x_k - root| <= |F(x_k)|/(1-e), inside Newton's quadratic range, so two
// steps bring it to rounding (at e = 0.9999, 1e-9 -> 5e-15 -> 1e-25).  The
// state is then the root, as the converged reference has it, rather than x_k,
// whose phase may be off by up to ftol/(1-e) per drift.
//
// Returns the root and, in (s, m), its sine and cosine minus one.  A lane's
// (s, m) are fixed in the step where it stops, like its root: from the values
// at the point x of that step (c = 1 + m) and the step's correction d (the
// root is x - d), the first-order rotation
//   sin(x - d) = s - c d,  cos(x - d) - 1 = m + s d
// leaves out s d^2/2 and c d^3/6 (and their cosine counterparts): with
// |d| <= 2^-28 and Q >= 2^-24 (kepler_bound's floor) these stay below 0.05 ulp
// of the values and of x.  Lanes still iterating when the step budget runs
// out get sin/cos of their last iterate afresh; lanes that start with done
// set get (0, 0) (their xk is 0).  Each lane's values depend only on its own
// iterates, whichever lanes share its wavefront.  om = 1 - ec.
constexpr int KEPLER_EXTRA = 2;

template <bool SHORT>
TPM_DEV double kepler_newton(double ec, double es, double om, double dM, int kiters, double Q,
                             bool done, double xk, double& s, double& m, double& Fk) {
  bool converged = false;   // wave-uniform: every lane stopped
  s = 0.0;
  m = 0.0;
  Fk = 0.0;
  for (int it = 0; it < kiters + KEPLER_EXTRA; ++it) {
    if (it >= 1 && wave_all(done)) {
      converged = true;
      break;
    }
    double sv, mv;
    sincos_it<SHORT>(xk, sv, mv);
    double F = fma_(-ec, sv, fma_(-es, mv, xk - dM));
    if (it == kiters) Fk = done ? 0.0 : F;
    double Fp = fma_(-ec, mv, fma_(es, sv, om));
    double xn = fma_(-F, rcp_newton(Fp), xk);
    const double d = xk - xn;
    const double ad = __builtin_fabs(d), ax = __builtin_fabs(xn);
    bool small = (ad <= 0x1p-30 * ax) |
                 ((ad <= 0x1p-28) & (fma_(Q * ad, ad, -0x1p-54 * ax) <= 0.0));
    const double sn = fma_(-(1.0 + mv), d, sv), mn = fma_(sv, d, mv);
    s = done ? s : sn;
    m = done ? m : mn;
    xk = done ? xk : xn;
    done = done | small;
  }
  if (!converged) {
    double sf, mf;
    sincos_it<SHORT>(xk, sf, mf);
    s = done ? s : sf;
    m = done ? m : mf;
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
TPM_DEV double planet_newton(double ec, double es, double om, double dM, bool idle, double xk,
                             double& s, double& m) {
  bool done = idle;
  for (int it = 0; it < 40; ++it) {
    if (it >= 2 && wave_all(done)) return xk;
    double sv, mv;
    sincos_it<SHORT>(xk, sv, mv);
    const double F = fma_(-ec, sv, fma_(-es, mv, xk - dM));
    const double Fp = fma_(-ec, mv, fma_(es, sv, om));
    const double xn = fma_(-F, rcp_newton(Fp), xk);
    const double d = xk - xn;
    done = idle | (__builtin_fabs(d) <= 0x1p-30 * __builtin_fabs(xn));
    s = fma_(-(1.0 + mv), d, sv);
    m = fma_(sv, d, mv);
    xk = xn;
  }
  sincos_it<SHORT>(xk, s, m);
  return xk;
}

// The planet map's branch-free step (see the fast blocks of the planet map):
// exactly two Newton steps in the short sin/cos range, the same arithmetic as
// planet_newton<true> takes when it leaves after its second step.  `conv` is
// what that exit requires of the lane (idle, or a second correction of at
// most 2^-30 |x|); where it is false on any lane, planet_newton would have
// gone on and the caller redoes the step on the general path.
TPM_DEV double planet_newton2(double ec, double es, double om, double dM, bool idle, double xk,
                              double& s, double& m, bool& conv) {
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double sv, mv;
    sincos_it<true>(xk, sv, mv);
    const double F = fma_(-ec, sv, fma_(-es, mv, xk - dM));
    const double Fp = fma_(-ec, mv, fma_(es, sv, om));
    const double xn = fma_(-F, rcp_newton(Fp), xk);
    const double d = xk - xn;
    conv = idle | (__builtin_fabs(d) <= 0x1p-30 * __builtin_fabs(xn));
    s = fma_(-(1.0 + mv), d, sv);
    m = fma_(sv, d, mv);
    xk = xn;
  }
  return xk;
}

// Starter of the particles' Newton solve: with p = 1 - ec and t = dM/p, the
// series root of F = 0 through third order in t,
//   x0 = t - (es/(2p)) t^2 + (es^2/(2p^2) - ec/(6p)) t^3
// (F = p x + (es/2) x^2 + (ec/6) x^3 - dM + O(x^4)), clamped to dM +- w,
// w = 2(|ec| + |es|) (a bracket of the root).  Its error is O(e t^4): on
// near-circular orbits one Newton step from it is converged to rounding.
TPM_DEV double kepler_starter(double ec, double es, double om, double dM, double w) {
  const double oinv = rcp_newton(om);   // a first guess only (om = 1 - ec)
  const double t = dM * oinv;
  const double h = 0.5 * es * oinv;
  const double c3 = oinv * fma_(es, h, ec * (-1.0 / 6.0));
  const double x0 = t * fma_(t, fma_(c3, t, -h), 1.0);
  return __builtin_fmin(__builtin_fmax(x0, dM - w), dM + w);
}

// Q of kepler_newton's stopping rule from w = 2(|ec| + |es|): rounded up (the
// hardware reciprocal is good to 2^-24) and at least 2^-24; +inf where
// eb = w/2 > 0.75 (or NaN), which leaves those lanes the relative rule alone.
TPM_DEV double kepler_bound(double w) {
  const double eb = 0.5 * w;
  const double om = 1.0 - eb, op = 1.0 + eb;
  const double Q = (0.5 + 0x1p-20) * eb * (op * op) * __builtin_amdgcn_rcp(om * om * om);
  return eb <= 0.75 ? __builtin_fmax(Q, 0x1p-24) : __builtin_inf();
}

// The particles' Newton solve from the starter xk, with sin/cos of its result
// and F(x_k) of the fixed count (see kepler_newton).  (Each sin/cos decides its
// short path by itself: one copy of the loop keeps the particle kernel's
// registers within budget.)
TPM_DEV double kepler_solve(double ec, double es, double om, double dM, int kiters, double w,
                            double xk, double& s, double& m, double& Fk) {
  return kepler_newton<false>(ec, es, om, dM, kiters, kepler_bound(w), false, xk, s, m, Fk);
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
  const double w = 2.0 * (__builtin_fabs(ec) + __builtin_fabs(es));
  const double om = 1.0 - ec;
  double xk = kepler_starter(ec, es, om, dM, w);
  double s, m, Fk;
  xk = kepler_solve(ec, es, om, dM, kiters, w, xk, s, m, Fk);
  double F = fma_(-ec, s, fma_(-es, m, xk - dM));
  double Fp = fma_(-ec, m, fma_(es, s, om));
  // one compare: an unbound orbit counts as an infinite residual; the larger
  // of the fixed count's residual and the final one decides
  const double Fm = __builtin_fmax(__builtin_fabs(F), __builtin_fabs(Fk));
  const bool ok = (bound ? Fm : __builtin_inf()) <= ftol;
  double r1 = a * Fp;
  double r1inv = rcp(r1);
  double f = fma_(a * rinv, m, 1.0);
  double g = fma_(s - xk, ninv, dte);
  double fd = -(a * a) * n * s * rinv * r1inv;
  double gd = fma_(a * r1inv, m, 1.0);
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
// FAST: no wave-uniform branch; two Newton steps in the short sin/cos range
// (planet_newton2).  `bad` is set on a lane where the general form would have
// taken another path (the short range not allowed, or more Newton steps); the
// results are the general form's bit for bit where no lane of the wavefront
// is bad.  The general form leaves `bad` false.
template <bool FAST>
TPM_DEV bool drift_converged_t(const KepConst& K, double dt, bool lane_on,
                               double& x, double& y, double& z,
                               double& vx, double& vy, double& vz, bool& bad) {
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
  const double om = 1.0 - ec;
  double oinv = rcp_newton(om);   // a first guess only: one refinement is enough
  double t = dM * oinv;
  double xk = t * fma_(-0.5 * es * t, oinv, 1.0);
  double w = 2.0 * (__builtin_fabs(ec) + __builtin_fabs(es));
  xk = __builtin_fmin(__builtin_fmax(xk, dM - w), dM + w);
  double s, m;
  if (FAST) {
    bool conv;
    xk = planet_newton2(ec, es, om, dM, idle, xk, s, m, conv);
    bad = !(idle | short_args(dM, w)) | !conv;
  } else {
    bad = false;
    if (wave_all(idle | short_args(dM, w)))
      xk = planet_newton<true>(ec, es, om, dM, idle, xk, s, m);
    else
      xk = planet_newton<false>(ec, es, om, dM, idle, xk, s, m);
  }
  double Fp = fma_(-ec, m, fma_(es, s, om));
  double r1 = a * Fp;
  double r1inv = rcp(r1);
  double f = fma_(a * rinv, m, 1.0);
  double g = fma_(s - xk, ninv, dte);
  double fd = -(a * a) * n * s * rinv * r1inv;
  double gd = fma_(a * r1inv, m, 1.0);
  double nx = fma_(f, x, g * vx), ny = fma_(f, y, g * vy), nz = fma_(f, z, g * vz);
  double nvx = fma_(fd, x, gd * vx), nvy = fma_(fd, y, gd * vy), nvz = fma_(fd, z, gd * vz);
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return bound;
}

TPM_DEV bool drift_converged(const KepConst& K, double dt, bool lane_on,
                             double& x, double& y, double& z,
                             double& vx, double& vy, double& vz) {
  bool bad;
  return drift_converged_t<false>(K, dt, lane_on, x, y, z, vx, vy, vz, bad);
}

}  // namespace tpm
