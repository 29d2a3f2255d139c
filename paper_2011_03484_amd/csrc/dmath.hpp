// FP64 device math for gfx950: reciprocal, reciprocal square root and sin/cos,
// free of lane-divergent branches, so every lane of a wavefront runs the same
// instructions.
//
// * rcp / rsqrt start from the hardware approximations (v_rcp_f64, v_rsq_f64,
//   relative error below 2^-24 on gfx950) and correct them with fused
//   multiply-adds.  From the residual e of the estimate y (e = 1 - x y for a
//   reciprocal, e = 1 - x y^2 for a reciprocal square root) the exact value is
//   y / (1 - e) resp. y / sqrt(1 - e); the Taylor series of these in e,
//   truncated after e^2, leave an error of order e^3 < 2^-69, far below the
//   rounding of the last operations.  A Newton step (one FMA pair) is the
//   series truncated after e, good to about 2^-46.
// * sincos reduces the argument by pi/2 with the two-constant Cody-Waite scheme
//   done in fused multiply-adds (exact first product for the quadrant counts
//   used here, |q| <= 2^20), then evaluates the Taylor series of sin and of
//   cos - 1 on [-pi/4, pi/4] (truncation below 1e-19) in Estrin's form and
//   picks the quadrant with selects; a wavefront whose arguments are all
//   inside [-0.78, 0.78] skips the reduction (same values).
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

// True when p holds on every active lane: the ballot of p is the lane mask a
// vector compare already produced, so the test is a scalar compare against
// exec (no round trip of the predicate through a vector register).
TPM_DEV bool wave_all(bool p) {
  return __builtin_amdgcn_ballot_w64(p) == __builtin_amdgcn_read_exec();
}

// 1/x to rounding: y (1 + e + e^2), e = 1 - x y.
TPM_DEV double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma_(-x, y, 1.0);
  return fma_(y, fma_(e, e, e), y);
}

// 1/x good to about 2^-46 relative: enough inside a Newton iteration whose
// next step corrects the error.
TPM_DEV double rcp_newton(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma_(-x, y, 1.0);
  return fma_(y, e, y);
}

// 1/sqrt(x) for x > 0 to rounding: y (1 + e/2 + 3 e^2/8), e = 1 - x y^2
// (measured on gfx950 over 4M arguments spanning 1e-12..1e12: at most
// 1.5 * 2^-53 relative).
TPM_DEV double rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma_(-x, y * y, 1.0);
  return fma_(y * e, fma_(e, 0.375, 0.5), y);
}

// m / x^(3/2) for x > 0 (a force factor m/|d|^3 with x = |d|^2), from the same
// residual: m y^3 (1 + 3e/2 + 15 e^2/8), e = 1 - x y^2 (measured: at most
// 2.5 * 2^-53 relative; the cube of rsqrt reaches 6.9 * 2^-53).  c15 is the
// series' 3/2, which a caller may pass from a register it keeps for the
// purpose (see vgpr_held; the value, and so the result, is the same).
TPM_DEV double mul_rsqrt3(double m, double x, double c15 = 1.5) {
  double y = __builtin_amdgcn_rsq(x);
  double y2 = y * y;
  double e = fma_(-x, y2, 1.0);
  double mm = m * (y2 * y);
  return fma_(mm * e, fma_(e, 1.875, c15), mm);
}

// A value held in a VGPR: the compiler cannot turn it back into a constant.
// An FP64 instruction reads at most one scalar operand, so a constant that
// meets another scalar operand in one instruction is otherwise copied into a
// VGPR at every use.
TPM_DEV double vgpr_held(double v) {
  asm volatile("" : "+v"(v));
  return v;
}

// m / x^(3/2) with the series truncated after e: relative error below
// (15/8) e^2 < 2^-45; used where the result only scales a small perturbation.
TPM_DEV double mul_rsqrt3_1(double m, double x) {
  double y = __builtin_amdgcn_rsq(x);
  double y2 = y * y;
  double e = fma_(-x, y2, 1.0);
  double mm = m * (y2 * y);
  return fma_(mm * e, 1.5, mm);
}

// sqrt(x) and 1/sqrt(x) together for x > 0: rs = rsqrt(x), then one Newton
// correction of s = x rs against x.
TPM_DEV void sqrt_rsqrt(double x, double& s, double& rs) {
  rs = rsqrt(x);
  const double g = x * rs;
  s = fma_(fma_(-g, g, x), 0.5 * rs, g);
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

// sin r and cos r - 1 for |r| <= pi/4 (plus a little slack).  With z = r^2
// the two series in z are evaluated in Estrin's pairing (shared z^2, z^4),
// which halves the dependent-FMA depth of Horner's rule at the same count.
// cos r - 1 = -z/2 + z^2 (C4 + C6 z + ...) is summed as such, never as cos r
// minus 1: the f and g functions and Kepler's equation need it for small r,
// where the difference would carry the rounding of cos r (half an ulp of 1)
// into a value far below 1.
TPM_DEV void sincos_poly(double r, double& s, double& m) {
  const double z = r * r;
  const double z2 = z * z;
  const double z4 = z2 * z2;
  // sin r = r + r z (S3 + S5 z + ... + S17 z^7)
  double s01 = fma_(S5, z, S3), s23 = fma_(S9, z, S7);
  double s45 = fma_(S13, z, S11), s67 = fma_(S17, z, S15);
  double ps = fma_(z4, fma_(z2, s67, s45), fma_(z2, s23, s01));
  s = fma_(r * z, ps, r);
  // cos r - 1 = -z/2 + z^2 (C4 + C6 z + ... + C18 z^7)
  double c01 = fma_(C6, z, C4), c23 = fma_(C10, z, C8);
  double c45 = fma_(C14, z, C12), c67 = fma_(C18, z, C16);
  double pc = fma_(z4, fma_(z2, c67, c45), fma_(z2, c23, c01));
  m = fma_(z2, pc, -0.5 * z);
}

// sincos_poly by Horner's rule: fewer instructions, longer dependency chains.
// The planet map's lone wavefront runs it faster (its time is its instruction
// count); the particle kernels, with many wavefronts per SIMD, prefer Estrin's
// shorter chains.  The values agree to rounding.
TPM_DEV void sincos_poly_horner(double r, double& s, double& m) {
  const double z = r * r;
  double ps = fma_(S17, z, S15);
  ps = fma_(ps, z, S13);
  ps = fma_(ps, z, S11);
  ps = fma_(ps, z, S9);
  ps = fma_(ps, z, S7);
  ps = fma_(ps, z, S5);
  ps = fma_(ps, z, S3);
  s = fma_(r * z, ps, r);
  double pc = fma_(C18, z, C16);
  pc = fma_(pc, z, C14);
  pc = fma_(pc, z, C12);
  pc = fma_(pc, z, C10);
  pc = fma_(pc, z, C8);
  pc = fma_(pc, z, C6);
  pc = fma_(pc, z, C4);
  m = fma_(z * z, pc, -0.5 * z);
}

// sin(x), cos(x) and cos(x) - 1 for |x| up to about 2^20.  When every active
// lane of the wavefront has |x| <= 0.78 (< pi/4, so the quadrant count is 0
// and the reduction leaves x unchanged) the reduction is skipped; the values
// are the same (the full path would only turn a -0 input into +0).  The only
// branch is that wave-uniform one.  cos(x) - 1 comes from the series in the
// first quadrant; beyond it |cos(x) - 1| >= 1 - cos(pi/4) and the difference
// loses at most two bits.
TPM_DEV void sincos3(double x, double& s, double& c, double& m) {
  if (wave_all(__builtin_fabs(x) <= 0.78)) {
    sincos_poly(x, s, m);
    c = 1.0 + m;
    return;
  }
  double q = __builtin_rint(x * TWO_OVER_PI);
  double r = fma_(-q, PIO2_HI, x);
  r = fma_(-q, PIO2_LO, r);
  double ps, pm;
  sincos_poly(r, ps, pm);
  const double pc = 1.0 + pm;
  int iq = (int)q;
  bool swap = iq & 1;
  double ss = swap ? pc : ps;
  double cc = swap ? ps : pc;
  s = (iq & 2) ? -ss : ss;
  c = ((iq + 1) & 2) ? -cc : cc;
  m = (iq & 3) == 0 ? pm : c - 1.0;
}

// sin(x) and cos(x) - 1 (see sincos3).
TPM_DEV void sincosm1(double x, double& s, double& m) {
  double c;
  sincos3(x, s, c, m);
}

// sin(x) and cos(x) (see sincos3).
TPM_DEV void sincos(double x, double& s, double& c) {
  double m;
  sincos3(x, s, c, m);
}

}  // namespace tpm
