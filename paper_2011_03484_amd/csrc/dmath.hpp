// FP64 device math for gfx950: reciprocal, reciprocal square root and sin/cos,
// all branch-free so that every lane of a wavefront runs the same instructions.
//
// * rcp / rsqrt start from the hardware approximations (v_rcp_f64, v_rsq_f64,
//   about 23 good bits) and refine them by Newton-Raphson with fused
//   multiply-adds; each refinement doubles the number of good bits.
// * sincos reduces the argument by pi/2 with the two-constant Cody-Waite scheme
//   done in fused multiply-adds (exact first product for the quadrant counts
//   used here, |q| <= 2^20), then evaluates the Taylor series of sin and cos on
//   [-pi/4, pi/4] (truncation below 1e-19) and picks the quadrant with selects.
//   The constants are pi/2 split into its nearest double and the nearest double
//   to the remainder (from 50-digit pi; gen_constants.py reproduces them) and
//   the reciprocals 1/n! of the Taylor series.
//
// Every floating-point expression is written with explicit fma() so results do
// not depend on the compiler's contraction choices (sources are compiled with
// -ffp-contract=off): the same inputs give the same bits in every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpm {

#define TPM_DEV __device__ __forceinline__

TPM_DEV double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x, error about 1 ulp (two refinements of the hardware estimate).
TPM_DEV double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma_(-x, y, 1.0);
  y = fma_(y, e, y);
  e = fma_(-x, y, 1.0);
  return fma_(y, e, y);
}

// 1/x good to about 2^-46 relative: enough inside a Newton iteration whose
// next step corrects the error.
TPM_DEV double rcp_newton(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma_(-x, y, 1.0);
  return fma_(y, e, y);
}

// 1/sqrt(x) for x > 0, error about 1 ulp.  Coupled iteration on
// g ~ sqrt(x), h ~ 1/(2 sqrt(x)):  r = 1/2 - g h;  g += g r;  h += h r.
TPM_DEV double rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  double r = fma_(-g, h, 0.5);
  g = fma_(g, r, g);
  h = fma_(h, r, h);
  r = fma_(-g, h, 0.5);
  h = fma_(h, r, h);
  return h + h;
}

// sqrt(x) and 1/sqrt(x) together for x > 0.
TPM_DEV void sqrt_rsqrt(double x, double& s, double& rs) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  double r = fma_(-g, h, 0.5);
  g = fma_(g, r, g);
  h = fma_(h, r, h);
  r = fma_(-g, h, 0.5);
  g = fma_(g, r, g);
  h = fma_(h, r, h);
  // one last residual correction of g against x
  double d = fma_(-g, g, x);
  s = fma_(d, h, g);
  rs = h + h;
}

// pi/2 = PIO2_HI + PIO2_LO (nearest double, then nearest double to the rest)
constexpr double PIO2_HI = 0x1.921fb54442d18p+0;
constexpr double PIO2_LO = 0x1.1a62633145c07p-54;
constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;

// Taylor coefficients 1/n! with alternating signs
constexpr double S3 = -1.0 / 6.0;
constexpr double S5 = 1.0 / 120.0;
constexpr double S7 = -1.0 / 5040.0;
constexpr double S9 = 1.0 / 362880.0;
constexpr double S11 = -1.0 / 39916800.0;
constexpr double S13 = 1.0 / 6227020800.0;
constexpr double S15 = -1.0 / 1307674368000.0;
constexpr double S17 = 1.0 / 355687428096000.0;
constexpr double C4 = 1.0 / 24.0;
constexpr double C6 = -1.0 / 720.0;
constexpr double C8 = 1.0 / 40320.0;
constexpr double C10 = -1.0 / 3628800.0;
constexpr double C12 = 1.0 / 479001600.0;
constexpr double C14 = -1.0 / 87178291200.0;
constexpr double C16 = 1.0 / 20922789888000.0;
constexpr double C18 = -1.0 / 6402373705728000.0;

// sin and cos of r for |r| <= pi/4 (plus a little slack).
TPM_DEV void sincos_poly(double r, double& s, double& c) {
  double r2 = r * r;
  double ps = fma_(r2, S17, S15);
  ps = fma_(r2, ps, S13);
  ps = fma_(r2, ps, S11);
  ps = fma_(r2, ps, S9);
  ps = fma_(r2, ps, S7);
  ps = fma_(r2, ps, S5);
  ps = fma_(r2, ps, S3);
  s = fma_(r * r2, ps, r);
  double pc = fma_(r2, C18, C16);
  pc = fma_(r2, pc, C14);
  pc = fma_(r2, pc, C12);
  pc = fma_(r2, pc, C10);
  pc = fma_(r2, pc, C8);
  pc = fma_(r2, pc, C6);
  pc = fma_(r2, pc, C4);
  // cos = 1 - r2/2 + r2^2 pc, with the rounding of 1 - r2/2 carried along
  double hr = 0.5 * r2;
  double w = 1.0 - hr;
  double tail = (1.0 - w) - hr;
  c = w + fma_(r2 * r2, pc, tail);
}

// sin(x), cos(x) for |x| up to about 2^20, no branches.
TPM_DEV void sincos(double x, double& s, double& c) {
  double q = __builtin_rint(x * TWO_OVER_PI);
  double r = fma_(-q, PIO2_HI, x);
  r = fma_(-q, PIO2_LO, r);
  double ps, pc;
  sincos_poly(r, ps, pc);
  int iq = (int)q;
  bool swap = iq & 1;
  double ss = swap ? pc : ps;
  double cc = swap ? ps : pc;
  s = (iq & 2) ? -ss : ss;
  c = ((iq + 1) & 2) ? -cc : cc;
}

}  // namespace tpm
