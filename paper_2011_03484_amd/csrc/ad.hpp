// Derivatives of the test-particle map: forward (tangent) and reverse
// (adjoint) mode, by hand, for gfx950.
//
// One step of the map is kick(h) o drift(dt) o kick(h) with h = dt/2.
//  * Kick: v' = v + h a(r), a(r) = h0 - sum_j mu_j d_j/|d_j|^3, d_j = r - r_j.
//    Its Jacobian is [[I, 0], [h A, I]] with the symmetric
//    A = da/dr = sum_j mu_j (3 d_j d_j^T/|d_j|^5 - I/|d_j|^3); h0 and the planet
//    positions do not depend on the particle.
//  * Drift: the f-g Kepler drift (see kepler.hpp).  The change x of eccentric
//    anomaly is an implicit function of (ec, es, dM) through
//    x - ec sin x + es (1 - cos x) = dM, so by the implicit-function theorem
//    dx = (sin x dec - (1 - cos x) des + d dM) / F'(x).  Every other quantity
//    is an explicit expression; they are differentiated in order (tangent) or
//    in reverse order (adjoint).
// The fixed-count Newton iterate x_k stands for the root (its residual is
// below the Kepler-failure threshold), so derivatives are those of the exact
// drift at the computed state.  A particle removed at step n keeps its state,
// so nothing after step n contributes to its derivative.
#pragma once
#include "particle.hpp"

namespace tpm {

// Values of one drift that its derivatives need.
struct DriftVals {
  double u, r0, rinv, alpha, sa, a, n, ec, es, dMr, q, x, s, c, m, Fp, r1, f, g, fd, gd;
  double rsa, ninv, r1inv;   // 1/sa, 1/n, 1/r1 (the derivatives multiply by these)
  bool ok;
};

// Same arithmetic as drift_fixed (the particle kernel's drift), keeping the
// intermediate values; writes the drifted state only where ok.  KNOWN: the
// root of Kepler's equation and its sin and cos - 1 are given (kx, ks, km:
// the values an earlier evaluation of the same drift found), so the solve is
// skipped and every other value comes out bit for bit as that evaluation's.
template <bool KNOWN>
TPM_DEV void drift_vals_t(const KepConst& K, double dt, int kiters, double ftol, double x, double y,
                          double z, double vx, double vy, double vz, DriftVals& D, double& nx,
                          double& ny, double& nz, double& nvx, double& nvy, double& nvz,
                          double kx, double ks, double km) {
  double r2 = fma_(x, x, fma_(y, y, z * z));
  double v2 = fma_(vx, vx, fma_(vy, vy, vz * vz));
  double u = fma_(x, vx, fma_(y, vy, z * vz));
  D.u = u;
  sqrt_rsqrt(r2, D.r0, D.rinv);
  D.alpha = fma_(-v2, K.inv_mu, 2.0 * D.rinv);
  bool bound = D.alpha > 0.0;
  double rsa;
  sqrt_rsqrt(D.alpha, D.sa, rsa);
  D.rsa = rsa;
  double a = rsa * rsa;
  D.a = fma_(a, fma_(-D.alpha, a, 1.0), a);
  D.n = K.sqrt_mu * D.sa * D.alpha;
  double ninv = K.inv_sqrt_mu * rsa * D.a;
  D.ninv = ninv;
  D.ec = fma_(-D.r0, D.alpha, 1.0);
  D.es = u * D.sa * K.inv_sqrt_mu;
  double dM = D.n * dt;
  D.q = __builtin_rint(dM * INV_TWO_PI);
  double dMr = fma_(-D.q, TWO_PI_HI, dM);
  D.dMr = fma_(-D.q, TWO_PI_LO, dMr);
  double dte = (D.q == 0.0) ? dt : D.dMr * ninv;
  dM = D.dMr;
  const double om = 1.0 - D.ec;
  double xk, s, m, Fk;
  if (KNOWN) {
    xk = kx; s = ks; m = km; Fk = 0.0;
  } else {
    const double w = 2.0 * (__builtin_fabs(D.ec) + __builtin_fabs(D.es));
    xk = kepler_starter(D.ec, D.es, om, dM, w);
    xk = kepler_solve(D.ec, D.es, om, dM, kiters, w, xk, s, m, Fk);
  }
  double F = fma_(-D.ec, s, fma_(-D.es, m, xk - dM));
  D.Fp = fma_(-D.ec, m, fma_(D.es, s, om));
  D.ok = bound && (__builtin_fmax(__builtin_fabs(F), __builtin_fabs(Fk)) <= ftol);
  D.x = xk; D.s = s; D.m = m; D.c = 1.0 + m;
  D.r1 = D.a * D.Fp;
  double r1inv = rcp(D.r1);
  D.r1inv = r1inv;
  D.f = fma_(D.a * D.rinv, m, 1.0);
  D.g = fma_(s - xk, ninv, dte);
  D.fd = -(D.a * D.a) * D.n * s * D.rinv * r1inv;
  D.gd = fma_(D.a * r1inv, m, 1.0);
  nx = fma_(D.f, x, D.g * vx); ny = fma_(D.f, y, D.g * vy); nz = fma_(D.f, z, D.g * vz);
  nvx = fma_(D.fd, x, D.gd * vx); nvy = fma_(D.fd, y, D.gd * vy); nvz = fma_(D.fd, z, D.gd * vz);
}

TPM_DEV void drift_vals(const KepConst& K, double dt, int kiters, double ftol, double x, double y,
                        double z, double vx, double vy, double vz, DriftVals& D, double& nx,
                        double& ny, double& nz, double& nvx, double& nvy, double& nvz) {
  drift_vals_t<false>(K, dt, kiters, ftol, x, y, z, vx, vy, vz, D, nx, ny, nz, nvx, nvy, nvz, 0.0,
                      0.0, 0.0);
}

// Tangent of the drift: (dr, dv) at (r, v) -> (dr', dv').
TPM_DEV void drift_jvp(const KepConst& K, double dt, const DriftVals& D, const double r[3],
                       const double v[3], const double dr[3], const double dv[3], double odr[3],
                       double odv[3]) {
  double dr2 = 2.0 * (r[0] * dr[0] + r[1] * dr[1] + r[2] * dr[2]);
  double dv2 = 2.0 * (v[0] * dv[0] + v[1] * dv[1] + v[2] * dv[2]);
  double du = r[0] * dv[0] + r[1] * dv[1] + r[2] * dv[2] + v[0] * dr[0] + v[1] * dr[1] + v[2] * dr[2];
  double dr0 = 0.5 * dr2 * D.rinv;
  double drinv = -dr0 * D.rinv * D.rinv;
  double dalpha = 2.0 * drinv - dv2 * K.inv_mu;
  // divisions are multiplications by the reciprocals the drift computed
  // (1/a by alpha, 1/rinv by r0: equal to rounding)
  const double iFp = rcp(D.Fp), in2 = D.ninv * D.ninv;
  double dsa = 0.5 * dalpha * D.rsa;
  double da = -D.a * D.a * dalpha;
  double dn = K.sqrt_mu * (dsa * D.alpha + D.sa * dalpha);
  double dec = -(dr0 * D.alpha + D.r0 * dalpha);
  double des = (du * D.sa + D.u * dsa) * K.inv_sqrt_mu;
  double ddM = dn * dt;
  double ddte = (D.q == 0.0) ? 0.0 : (ddM * D.n - D.dMr * dn) * in2;
  double dx = (D.s * dec + D.m * des + ddM) * iFp;
  double ds = D.c * dx, dc = -D.s * dx;
  double dFp = -(dec * D.c + D.ec * dc) + des * D.s + D.es * ds;
  double df = (da * D.rinv + D.a * drinv) * D.m + D.a * D.rinv * dc;
  double dg = ddte + (ds - dx) * D.ninv - (D.s - D.x) * dn * in2;
  double dr1 = da * D.Fp + D.a * dFp;
  // fd = -s Q with Q = a^2 n rinv / r1
  double Q = D.a * D.a * D.n * D.rinv * D.r1inv;
  double dQ = Q * (2.0 * da * D.alpha + dn * D.ninv + drinv * D.r0 - dr1 * D.r1inv);
  double dP = D.s * dQ + Q * ds;
  double dfd = -dP;
  double dgd = (da * D.r1inv - D.a * dr1 * (D.r1inv * D.r1inv)) * D.m + D.a * D.r1inv * dc;
  for (int k = 0; k < 3; ++k) {
    odr[k] = df * r[k] + D.f * dr[k] + dg * v[k] + D.g * dv[k];
    odv[k] = dfd * r[k] + D.fd * dr[k] + dgd * v[k] + D.gd * dv[k];
  }
}

// Adjoint of the drift: given (lr', lv') = dL/d(r', v'), return dL/d(r, v).
// The expression graph of drift_vals is walked backwards.
TPM_DEV void drift_vjp(const KepConst& K, double dt, const DriftVals& D, const double r[3],
                       const double v[3], const double lr1[3], const double lv1[3], double lr[3],
                       double lv[3]) {
  // r' = f r + g v, v' = fd r + gd v
  double bf = 0, bg = 0, bfd = 0, bgd = 0;
  for (int k = 0; k < 3; ++k) {
    bf += lr1[k] * r[k];
    bg += lr1[k] * v[k];
    bfd += lv1[k] * r[k];
    bgd += lv1[k] * v[k];
    lr[k] = D.f * lr1[k] + D.fd * lv1[k];
    lv[k] = D.g * lr1[k] + D.gd * lv1[k];
  }
  double ba = 0, bc = 0, bs = 0, bx = 0, bn = 0, brinv = 0, br1 = 0, bFp = 0, bec = 0, bes = 0;
  double bdte = 0, bdM = 0, bsa = 0, balpha = 0, bu = 0, br0 = 0, bv2 = 0, br2 = 0;
  // divisions are multiplications by the reciprocals the drift computed
  // (1/a by alpha, 1/rinv by r0: equal to rounding)
  const double iFp = rcp(D.Fp), in2 = D.ninv * D.ninv;
  // gd = 1 + (a/r1)(c - 1)
  ba += bgd * D.m * D.r1inv;
  bc += bgd * D.a * D.r1inv;
  br1 -= bgd * D.a * D.m * (D.r1inv * D.r1inv);
  // fd = -s Q, Q = a^2 n rinv / r1
  {
    double Q = D.a * D.a * D.n * D.rinv * D.r1inv;
    double bQ = -bfd * D.s;
    bs -= bfd * Q;
    ba += bQ * 2.0 * Q * D.alpha;
    bn += bQ * Q * D.ninv;
    brinv += bQ * Q * D.r0;
    br1 -= bQ * Q * D.r1inv;
  }
  // r1 = a Fp
  ba += br1 * D.Fp;
  bFp += br1 * D.a;
  // g = dte + (s - x)/n
  bdte += bg;
  bs += bg * D.ninv;
  bx -= bg * D.ninv;
  bn -= bg * (D.s - D.x) * in2;
  // f = 1 + a rinv (c - 1)
  ba += bf * D.rinv * D.m;
  brinv += bf * D.a * D.m;
  bc += bf * D.a * D.rinv;
  // Fp = 1 - ec c + es s
  bec -= bFp * D.c;
  bc -= bFp * D.ec;
  bes += bFp * D.s;
  bs += bFp * D.es;
  // s = sin x, c = cos x
  bx += bs * D.c - bc * D.s;
  // x(ec, es, dM): implicit function of x - ec sin x + es (1 - cos x) = dM
  bec += bx * D.s * iFp;
  bes += bx * D.m * iFp;
  bdM += bx * iFp;
  // dte = dMr / n when a whole period was removed (else dt itself)
  if (D.q != 0.0) {
    bdM += bdte * D.ninv;
    bn -= bdte * D.dMr * in2;
  }
  // dM = n dt (minus a constant)
  bn += bdM * dt;
  // es = u sa / sqrt(mu)
  bu += bes * D.sa * K.inv_sqrt_mu;
  bsa += bes * D.u * K.inv_sqrt_mu;
  // ec = 1 - r0 alpha
  br0 -= bec * D.alpha;
  balpha -= bec * D.r0;
  // n = sqrt(mu) sa alpha
  bsa += bn * K.sqrt_mu * D.alpha;
  balpha += bn * K.sqrt_mu * D.sa;
  // a = 1/alpha, sa = sqrt(alpha)
  balpha -= ba * D.a * D.a;
  balpha += bsa * 0.5 * D.rsa;
  // alpha = 2 rinv - v2/mu
  brinv += 2.0 * balpha;
  bv2 -= balpha * K.inv_mu;
  // rinv = 1/r0, r0 = sqrt(r2)
  br0 -= brinv * D.rinv * D.rinv;
  br2 += br0 * 0.5 * D.rinv;
  for (int k = 0; k < 3; ++k) {
    lr[k] += 2.0 * br2 * r[k] + bu * v[k];
    lv[k] += 2.0 * bv2 * v[k] + bu * r[k];
  }
}

// A w with A = da/dr at position r for one table row (symmetric, so it also
// serves the adjoint).
template <int NP, typename RowT>
TPM_DEV void accel_jac(const RowT& row, const PlanetConst<NP>& P, const double r[3],
                       const double w[3], double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double d[3] = {r[0] - row[3 * j + 0], r[1] - row[3 * j + 1], r[2] - row[3 * j + 2]};
    double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double inv = rsqrt(d2);
    double inv3 = inv * inv * inv;
    double inv5 = inv3 * inv * inv;
    double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
    for (int k = 0; k < 3; ++k) out[k] += P.mu[j] * (3.0 * inv5 * dw * d[k] - inv3 * w[k]);
  }
}

}  // namespace tpm
