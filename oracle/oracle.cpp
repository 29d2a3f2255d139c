// TEST INFRASTRUCTURE ONLY -- the plain, slow FP64 CPU oracle.
//
// Only the tests, the package's smoke check and the benchmark's CPU-baseline
// leg may load this library.  It shares no code, header, table or constant
// generator with the HIP path; it is compiled by g++ with -ffp-contract=off and
// without fast-math, so every operation is one IEEE-754 double rounding.
//
// What it computes (Zhang & Gladman, "GLISSE", New Astronomy 2021):
//   * sec. 2.2, eq. (H = H_Kepler + H_int): each test particle is advanced by the
//     Wisdom-Holman mixed-variable symplectic leapfrog -- half kick from H_int,
//     Kepler drift about the central mass for a full step, half kick.
//   * sec. 2.2, difference form of Kepler's equation: the drift solves
//     x - ec sin x + es (1 - cos x) = dM for the change x of eccentric anomaly
//     (ec = e cos E0, es = e sin E0) and applies the f and g functions.
//   * sec. 2.2, kick equation: dv/dt = h0 - sum_j mu_j (r - r_j)/|r - r_j|^3 with
//     the indirect term h0 = -sum_j mu_j r_j/|r_j|^3 (sec. 2.2, "common
//     heliocentric force").
//   * sec. 2.2: planets are integrated once with the standard Wisdom-Holman map
//     in Jacobi coordinates; every particle shares their positions.
//   * sec. 2.2, close-encounter paragraphs: a particle is frozen on close approach
//     (fixed distance or Hill multiple), recording which planet removed it; a
//     particle whose fixed-iteration Kepler solve does not converge is frozen too.
//
// Readings where the paper is silent (all listed in the design notes):
//   kick-drift-kick with planet rows at t_n and t_{n+1}; checks at every step
//   boundary on the synchronised state (r_n, v_n); precedence encounter > escape
//   > Kepler failure; lowest planet index wins; strict < and >; unbound drift or
//   |F(x_k)| > kepler_ftol after the fixed-k reference iteration -> Kepler
//   failure; dM reduced to (-pi, pi].
//
// The particle map is a template over the scalar type so the same code, run on
// std::complex<double>, yields the exact derivative of the discrete map by the
// complex-step method (Squire & Trapp 1998): every branch decides on real parts.
// The tangent, the state-transition matrix and the adjoint (its transpose) of
// the oracle all come from that.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <chrono>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

const double kTwoPi = 2.0 * M_PI;

// ---------------------------------------------------------------------------
// Operation count of the method's particle step (for the throughput roofline;
// nothing here changes a computed value).  Counted carries a double; while a
// count is on, each add, subtract and multiply is tallied, and each distinct
// reciprocal (x / y counts one reciprocal of y and one multiply), square root
// and sine-cosine pair once per stretch between restarts (count_boundary), so that
// values this plain source evaluates more than once (the three components of
// one force divided by one |d|^3; sin and cos of one Newton iterate in both F
// and F'; 1/mu in v^2/mu and alpha/mu) count once.  Negation and comparisons
// are free.
// ---------------------------------------------------------------------------
struct OpTally {
  int64_t add = 0, mul = 0, rcp = 0, sqrt = 0, sincos = 0;
  std::vector<double> rcp_seen, sqrt_seen, sc_seen;
  bool on = false;
  bool first(std::vector<double>& seen, double v) {
    for (double x : seen)
      if (x == v) return false;
    seen.push_back(v);
    return true;
  }
};
thread_local OpTally g_tally;

struct Counted {
  double v;
  Counted(double x = 0.0) : v(x) {}
};
inline double re(const Counted& x) { return x.v; }
inline Counted operator+(const Counted& a, const Counted& b) {
  if (g_tally.on) g_tally.add++;
  return a.v + b.v;
}
inline Counted operator-(const Counted& a, const Counted& b) {
  if (g_tally.on) g_tally.add++;
  return a.v - b.v;
}
inline Counted operator-(const Counted& a) { return -a.v; }
inline Counted operator*(const Counted& a, const Counted& b) {
  if (g_tally.on) g_tally.mul++;
  return a.v * b.v;
}
inline Counted operator/(const Counted& a, const Counted& b) {
  if (g_tally.on) {
    g_tally.mul++;
    if (g_tally.first(g_tally.rcp_seen, b.v)) g_tally.rcp++;
  }
  return a.v / b.v;
}
inline Counted& operator+=(Counted& a, const Counted& b) { return a = a + b; }

// sqrt, sin and cos of the templates below: the library routines for double
// and complex, the tallied forms for Counted.
template <class T>
inline T tsqrt(const T& x) { return std::sqrt(x); }
template <class T>
inline T tsin(const T& x) { return std::sin(x); }
template <class T>
inline T tcos(const T& x) { return std::cos(x); }
inline Counted tsqrt(const Counted& x) {
  if (g_tally.on && g_tally.first(g_tally.sqrt_seen, x.v)) g_tally.sqrt++;
  return std::sqrt(x.v);
}
inline Counted tsin(const Counted& x) {
  if (g_tally.on && g_tally.first(g_tally.sc_seen, x.v)) g_tally.sincos++;
  return std::sin(x.v);
}
inline Counted tcos(const Counted& x) {
  if (g_tally.on && g_tally.first(g_tally.sc_seen, x.v)) g_tally.sincos++;
  return std::cos(x.v);
}

// Each step, and each Newton iterate within it, is a new evaluation of the
// method, even where rounding repeats a value: the repeat tally restarts at
// each of them (a no-op for the other number types).
inline void count_boundary(const double&) {}
inline void count_boundary(const cplx&) {}
inline void count_boundary(const Counted&) {
  g_tally.rcp_seen.clear();
  g_tally.sqrt_seen.clear();
  g_tally.sc_seen.clear();
}

// The count follows the method, whose drift takes its state from the fixed-k
// iterate x_k; this oracle's own converged re-solve (kep_solve) is left out of
// it and the counted drift continues from x_k.
template <class T>
struct MethodOnly {
  static constexpr bool value = false;
};
template <>
struct MethodOnly<Counted> {
  static constexpr bool value = true;
};

enum { ACTIVE = 0, ENCOUNTER = 1, ESCAPE = 2, KEPLER = 3 };

// ---------------------------------------------------------------------------
// Kepler's equation in difference form (sec. 2.2):
//   F(x) = x - ec sin x + es (1 - cos x) - dM,  F'(x) = 1 - ec cos x + es sin x.
// Since ec sin x - es (1 - cos x) = e [sin(E0 + x) - sin E0], the root obeys
// |x - dM| <= 2e, and F' >= 1 - e > 0 makes it unique for e < 1.
// ---------------------------------------------------------------------------
// cos x - 1 as -2 sin^2(x/2), the same quantity without the cancellation of
// subtracting cos x from 1 when x is small (there c - 1 would carry the
// rounding of cos x, half an ulp of 1, into a value far below 1).  The tally
// follows the method's plain subtraction.
template <class T>
inline T cosm1(const T& x) {
  T h = tsin(0.5 * x);
  return -2.0 * h * h;
}
inline Counted cosm1(const Counted& x) { return tcos(x) - 1.0; }

template <class T>
inline T kep_F(const T& x, const T& ec, const T& es, const T& dM) {
  return x - ec * tsin(x) - es * cosm1(x) - dM;
}
template <class T>
inline T kep_dF(const T& x, const T& ec, const T& es) {
  return 1.0 - ec * tcos(x) + es * tsin(x);
}

// Fixed-k reference iteration (sec. 2.2: a fixed number of Newton iterations,
// five by default, from a starting guess the paper leaves to judgement).
// Starter: the series solution of F = 0 for small dM through third order.
// With p = 1 - ec and t = dM/p, F = p x + (es/2) x^2 + (ec/6) x^3 - dM + O(x^4)
// vanishes for x = t - (es/(2p)) t^2 + (es^2/(2p^2) - ec/(6p)) t^3 + O(t^4).
// It is clamped to the bracket dM +- 2(|ec| + |es|) (a valid bracket since
// |ec| + |es| >= e).  Returns x_k.
template <class T>
T kep_fixedk(const T& ec, const T& es, const T& dM, int k) {
  T om = 1.0 - ec;
  T t = dM / om;
  T q = es / om;
  T x = t - 0.5 * q * t * t + (0.5 * q * q - (1.0 / 6.0) * ec / om) * t * t * t;
  double w = 2.0 * (std::fabs(re(ec)) + std::fabs(re(es)));
  if (re(x) > re(dM) + w) x = dM + w;
  if (re(x) < re(dM) - w) x = dM - w;
  for (int i = 0; i < k; ++i) {
    count_boundary(x);
    x = x - kep_F(x, ec, es, dM) / kep_dF(x, ec, es);
  }
  count_boundary(x);
  return x;
}

// Converged solution: Newton safeguarded by bisection inside the bracket
// [dM - 2e, dM + 2e], stopped when a Newton correction is within 2 ulp of x,
// then one last Newton step (which also converges the imaginary part in the
// complex-step instantiation).
template <class T>
T kep_solve(const T& ec, const T& es, const T& dM, int* iters) {
  double e = std::sqrt(re(ec) * re(ec) + re(es) * re(es));
  double lo = re(dM) - 2.0 * e, hi = re(dM) + 2.0 * e;
  T x = kep_fixedk(ec, es, dM, 0);
  int it = 0;
  for (; it < 100; ++it) {
    T F = kep_F(x, ec, es, dM);
    if (re(F) == 0.0) break;
    if (re(F) < 0.0) lo = std::fmax(lo, re(x)); else hi = std::fmin(hi, re(x));
    T xn = x - F / kep_dF(x, ec, es);
    if (!(re(xn) > lo && re(xn) < hi)) {
      if (hi - lo <= 4.0 * std::ldexp(std::fabs(re(x)) + 1e-300, -52)) break;
      xn = T(0.5 * (lo + hi));
    }
    double dx = std::fabs(re(xn) - re(x));
    x = xn;
    if (dx <= 2.0 * std::ldexp(std::fabs(re(x)), -52)) break;
  }
  x = x - kep_F(x, ec, es, dM) / kep_dF(x, ec, es);
  if (iters) *iters = it;
  return x;
}

struct KepOut {
  int ok;
  double f, g, fd, gd;
};

// Two-body drift of (r, v) about a mass mu for time dt with the f and g
// functions (sec. 2.2, drift step; the element <-> Cartesian conversions of the
// paper's steps 2 and 4 are carried by f, g).  Returns 0 (and leaves r, v
// alone) when the orbit is unbound (alpha <= 0) or when the fixed-k reference
// iteration leaves |F(x_k)| > ftol (kfix < 0 skips that test).
template <class T>
int drift(double mu, T r[3], T v[3], double dt, int kfix, double ftol, KepOut* dbg = nullptr) {
  T r0 = tsqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  T u = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
  T alpha = 2.0 / r0 - v2 / mu;            // 1/a
  if (!(re(alpha) > 0.0)) return 0;
  T a = 1.0 / alpha;
  T n = tsqrt(mu * alpha) * alpha;         // sqrt(mu / a^3)
  T ec = 1.0 - r0 * alpha;                 // e cos E0
  T es = u * tsqrt(alpha / mu);            // e sin E0
  T dM = n * dt;
  T dte = dt;
  double q = std::rint(re(dM) / kTwoPi);
  if (q != 0.0) {                          // reduce dM to (-pi, pi]
    dM = dM - q * kTwoPi;
    dte = dM / n;
  }
  T xk = dM;
  if (kfix >= 0) {
    xk = kep_fixedk(ec, es, dM, kfix);
    if (!(std::fabs(re(kep_F(xk, ec, es, dM))) <= ftol)) return 0;
  }
  T x = MethodOnly<T>::value ? xk : kep_solve(ec, es, dM, nullptr);
  T s = tsin(x), c = tcos(x);
  T r1 = a * (1.0 - ec * c + es * s);
  T cm1 = cosm1(x);
  T f = 1.0 + (a / r0) * cm1;
  T g = dte + (s - x) / n;
  T fd = -(a * a * n * s) / (r1 * r0);
  T gd = 1.0 + (a / r1) * cm1;
  T rn[3], vn[3];
  for (int k = 0; k < 3; ++k) {
    rn[k] = f * r[k] + g * v[k];
    vn[k] = fd * r[k] + gd * v[k];
  }
  for (int k = 0; k < 3; ++k) { r[k] = rn[k]; v[k] = vn[k]; }
  if (dbg) { dbg->ok = 1; dbg->f = re(f); dbg->g = re(g); dbg->fd = re(fd); dbg->gd = re(gd); }
  return 1;
}

// ---------------------------------------------------------------------------
// Drift in universal variables, for orbits the elliptic solve above refuses
// (unbound, or not converged by the fixed-k iteration: near-parabolic); the
// paper names the high-eccentricity case as future work (sec. 2.2, Kepler
// solver paragraph).  Textbook two-body propagation valid for every conic:
// with sigma0 = r0.v0/sqrt(mu), alpha = 2/r0 - v0^2/mu and psi = alpha chi^2,
// the universal anomaly chi solves
//   F(chi) = r0 chi (1 - psi c3) + sigma0 chi^2 c2 + chi^3 c3 - sqrt(mu) dt = 0
// (equivalently r0 chi + sigma0 chi^2 c2 + (1 - alpha r0) chi^3 c3), whose
// derivative is the radius r(chi) = chi^2 c2 + sigma0 chi (1 - psi c3) +
// r0 (1 - psi c2) > 0; c2, c3 are the Stumpff functions.  Then f = 1 -
// chi^2 c2 / r0, g = dt - chi^3 c3 / sqrt(mu) (evaluated as (r0 chi (1 -
// psi c3) + sigma0 chi^2 c2) / sqrt(mu), the same by F = 0), fdot = sqrt(mu)
// chi (psi c3 - 1) / (r r0), gdot = 1 - chi^2 c2 / r.  F is increasing in chi, so the root
// is bracketed and found by Newton steps safeguarded by bisection.
// ---------------------------------------------------------------------------
// c2(psi) = (1 - cos sqrt psi)/psi, c3(psi) = (sqrt psi - sin sqrt psi)/psi^(3/2)
// (hyperbolic forms for psi < 0; their power series for |psi| < 1).
void stumpff(double psi, double& c2, double& c3) {
  if (std::fabs(psi) < 1.0) {
    double t2 = 0.5, t3 = 1.0 / 6.0;   // k = 0 terms 1/2!, 1/3!
    c2 = t2;
    c3 = t3;
    for (int k = 1; k <= 16; ++k) {
      t2 *= -psi / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
      t3 *= -psi / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
      c2 += t2;
      c3 += t3;
    }
  } else if (psi > 0.0) {
    const double sp = std::sqrt(psi);
    c2 = (1.0 - std::cos(sp)) / psi;
    c3 = (sp - std::sin(sp)) / (psi * sp);
  } else {
    const double sp = std::sqrt(-psi);
    c2 = (std::cosh(sp) - 1.0) / (-psi);
    c3 = (std::sinh(sp) - sp) / (-psi * sp);
  }
}

int drift_universal(double mu, double r[3], double v[3], double dt) {
  const double r0 = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double smu = std::sqrt(mu);
  const double sigma0 = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) / smu;
  const double alpha = 2.0 / r0 - v2 / mu;
  const double target = smu * dt;
  auto F = [&](double chi, double& rr, double& c2, double& c3) {
    const double psi = alpha * chi * chi;
    stumpff(psi, c2, c3);
    rr = chi * chi * c2 + sigma0 * chi * (1.0 - psi * c3) + r0 * (1.0 - psi * c2);
    return r0 * chi + sigma0 * chi * chi * c2 + (1.0 - alpha * r0) * chi * chi * chi * c3 - target;
  };
  if (dt == 0.0) return 1;
  double rr, c2, c3;
  // bracket: F(0) = -target; step outwards from chi = target / r0
  double lo = 0.0, hi = target / r0;
  for (int i = 0; i < 200 && (dt > 0 ? F(hi, rr, c2, c3) < 0.0 : F(hi, rr, c2, c3) > 0.0); ++i) {
    lo = hi;
    hi *= 2.0;
  }
  if (!std::isfinite(F(hi, rr, c2, c3))) return 0;
  if (dt < 0) std::swap(lo, hi);     // now F(lo) <= 0 <= F(hi), lo < hi
  double chi = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double Fv = F(chi, rr, c2, c3);
    if (Fv == 0.0) break;
    if (Fv < 0.0) lo = chi; else hi = chi;
    double cn = chi - Fv / rr;
    if (!(cn > lo && cn < hi)) cn = 0.5 * (lo + hi);
    const double d = std::fabs(cn - chi);
    chi = cn;
    if (d <= 2.0 * std::ldexp(std::fabs(chi), -52) || hi - lo <= 2.0 * std::ldexp(std::fabs(chi), -52))
      break;
  }
  F(chi, rr, c2, c3);
  const double psi = alpha * chi * chi;
  const double f = 1.0 - chi * chi * c2 / r0;
  // g = dt - chi^3 c3 / sqrt(mu), with dt replaced by its value from F = 0
  // (no cancellation near pericentre of a near-parabolic orbit)
  const double g = (r0 * chi * (1.0 - psi * c3) + sigma0 * chi * chi * c2) / smu;
  const double fd = smu * chi * (psi * c3 - 1.0) / (rr * r0);
  const double gd = 1.0 - chi * chi * c2 / rr;
  if (!(std::isfinite(f) && std::isfinite(g) && std::isfinite(fd) && std::isfinite(gd))) return 0;
  double rn[3], vn[3];
  for (int k = 0; k < 3; ++k) {
    rn[k] = f * r[k] + g * v[k];
    vn[k] = fd * r[k] + gd * v[k];
  }
  for (int k = 0; k < 3; ++k) { r[k] = rn[k]; v[k] = vn[k]; }
  return 1;
}

// The universal drift as the fallback of the particle step (double only; the
// derivative and operation-count instantiations never take it).
inline int universal_fallback(double mu, double* r, double* v, double dt) {
  return drift_universal(mu, r, v, dt);
}
template <class T>
int universal_fallback(double, T*, T*, double) { return 0; }

// ---------------------------------------------------------------------------
// Particle kick acceleration from one planet-table row (sec. 2.2 kick equation):
//   a = h0 - sum_j mu_j (r - r_j) / |r - r_j|^3.
// Also returns the lowest planet index j with |r - r_j| < rcrit_j, or -1.
// Row layout: r_1 (3), ..., r_np (3), h0 (3), heliocentric.
// ---------------------------------------------------------------------------
template <class T>
int kick_accel(const double* row, int np, const double* mu, const double* rcrit,
               const T r[3], T acc[3]) {
  int hit = -1;
  const double* h0 = row + 3 * np;
  for (int k = 0; k < 3; ++k) acc[k] = T(h0[k]);
  for (int j = 0; j < np; ++j) {
    T d[3];
    for (int k = 0; k < 3; ++k) d[k] = r[k] - row[3 * j + k];
    T d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    T dist = tsqrt(d2);
    if (hit < 0 && re(dist) < rcrit[j]) hit = j;
    T d3 = d2 * dist;
    for (int k = 0; k < 3; ++k) acc[k] = acc[k] - mu[j] * d[k] / d3;
  }
  return hit;
}

struct Deact {
  int64_t step;
  int32_t reason;
  int32_t planet;
};

// One particle through rows 0..nsteps of a table that starts at global step
// step0.  Checks run at every boundary on the synchronised state; on a hit the
// state of that boundary is kept.
// smp(n, row, r, v) is called at every boundary n = step0 + row that the
// particle passes while active (the diagnostics below; nothing by default).
struct NoSample {
  template <class T>
  void operator()(int64_t, int64_t, const T*, const T*) const {}
};

template <class T, class S = NoSample>
Deact run_particle(double mu0, int np, const double* mu, const double* rcrit, double rmax,
                   const double* table, int64_t nsteps, double dt, int64_t step0,
                   int kfix, double ftol, T r[3], T v[3], S&& smp = S(), bool universal = false) {
  const int rowlen = 3 * np + 3;
  const double h = 0.5 * dt;
  T acc[3];
  int hit = kick_accel(table, np, mu, rcrit, r, acc);
  auto escaped = [&](const T* rr) {
    T r2 = rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2];
    return rmax > 0.0 && re(tsqrt(r2)) > rmax;
  };
  if (hit >= 0) return {step0, ENCOUNTER, hit};
  if (escaped(r)) return {step0, ESCAPE, -1};
  smp(step0, 0, r, v);
  for (int64_t i = 0; i < nsteps; ++i) {
    count_boundary(r[0]);
    T rn[3], vn[3];
    for (int k = 0; k < 3; ++k) { rn[k] = r[k]; vn[k] = v[k] + h * acc[k]; }
    if (!drift(mu0, rn, vn, dt, kfix, ftol) &&
        !(universal && universal_fallback(mu0, rn, vn, dt)))
      return {step0 + i, KEPLER, -1};
    hit = kick_accel(table + (i + 1) * rowlen, np, mu, rcrit, rn, acc);
    for (int k = 0; k < 3; ++k) { r[k] = rn[k]; v[k] = vn[k] + h * acc[k]; }
    if (hit >= 0) return {step0 + i + 1, ENCOUNTER, hit};
    if (escaped(r)) return {step0 + i + 1, ESCAPE, -1};
    smp(step0 + i + 1, i + 1, r, v);
  }
  return {-1, ACTIVE, -1};
}

// ---------------------------------------------------------------------------
// Close-encounter hand-off (sec. 5: particles in close encounters move off the
// main integration to a separate treatment; the paper leaves the method open).
// Reading: at every step boundary n, a particle within r_enc,j of any planet
// takes its next step as an encounter step, any other particle the plain map
// step above.  An encounter step divides dt into M equal substeps of
// h = dt / M, each a kick - drift - kick of the same map:
//   v += (h/2) a(t_i);  Kepler drift about mu0 for h;  v += (h/2) a(t_i + h),
// with the planets between rows n and n+1 on the cubic Hermite interpolant of
// their heliocentric positions and velocities at the two rows (the row values
// themselves at the step's two ends), and h0 = -sum_j mu_j r_j / |r_j|^3 of
// the interpolated positions.  Removal: within r_rem,j of a planet at any step
// or substep boundary (lowest j; deact_step n at a step boundary n, n + 1 at a
// substep inside step n), beyond rmax at a step boundary, a refused drift (the
// state at the start of the failing substep, deact_step n).  At a boundary
// the order is: within r_rem, beyond rmax, then the mode of the next step.
// ---------------------------------------------------------------------------
// Planet j's heliocentric position at fraction tau of the step between rows a
// and b (positions ra, rb, velocities va, vb), by the cubic Hermite basis.
inline void hermite_at(double tau, double dt, const double* ra, const double* va,
                       const double* rb, const double* vb, double* out) {
  const double t2 = tau * tau, t3 = t2 * tau;
  const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
  const double h10 = t3 - 2.0 * t2 + tau;
  const double h01 = -2.0 * t3 + 3.0 * t2;
  const double h11 = t3 - t2;
  for (int c = 0; c < 3; ++c)
    out[c] = h00 * ra[c] + h10 * dt * va[c] + h01 * rb[c] + h11 * dt * vb[c];
}

// Acceleration of the particle at fraction tau of the step from row a (with
// its velocities va) to row b: a = h0 - sum_j mu_j (r - r_j)/|r - r_j|^3 with
// interpolated planets; returns the lowest j with |r - r_j| < rrem_j, or -1.
int interp_accel(double tau, double dt, int np, const double* mu, const double* rrem,
                 const double* rowa, const double* va, const double* rowb, const double* vb,
                 const double r[3], double acc[3]) {
  double pj[8][3];
  double h0[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < np; ++j) {
    hermite_at(tau, dt, rowa + 3 * j, va + 3 * j, rowb + 3 * j, vb + 3 * j, pj[j]);
    const double p2 = pj[j][0] * pj[j][0] + pj[j][1] * pj[j][1] + pj[j][2] * pj[j][2];
    const double p3 = p2 * std::sqrt(p2);
    for (int c = 0; c < 3; ++c) h0[c] -= mu[j] * pj[j][c] / p3;
  }
  for (int c = 0; c < 3; ++c) acc[c] = h0[c];
  int hit = -1;
  for (int j = 0; j < np; ++j) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = r[c] - pj[j][c];
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double dist = std::sqrt(d2);
    if (hit < 0 && dist < rrem[j]) hit = j;
    const double d3 = d2 * dist;
    for (int c = 0; c < 3; ++c) acc[c] -= mu[j] * d[c] / d3;
  }
  return hit;
}

// Lowest planet index with |r - r_j| < rad_j in a table row, or -1.
int within(const double* row, int np, const double* rad, const double r[3]) {
  for (int j = 0; j < np; ++j) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = r[c] - row[3 * j + c];
    if (std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < rad[j]) return j;
  }
  return -1;
}

// One particle through rows 0..nsteps (table, and planet velocities vtable
// [nsteps+1][np][3]) with the hand-off reading above; encounter_steps
// receives the number of encounter steps taken.
Deact run_particle_handoff(double mu0, int np, const double* mu, const double* renc,
                           const double* rrem, double rmax, const double* table,
                           const double* vtable, int64_t nsteps, double dt, int64_t step0,
                           int kfix, double ftol, bool universal, int M, double r[3], double v[3],
                           int64_t* encounter_steps) {
  const int rowlen = 3 * np + 3;
  const double h = dt / M;
  auto escaped = [&](const double* rr) {
    return rmax > 0.0 && std::sqrt(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]) > rmax;
  };
  auto drift_or_fallback = [&](double* rr, double* vv, double tau_dt) {
    return drift(mu0, rr, vv, tau_dt, kfix, ftol) != 0 ||
           (universal && universal_fallback(mu0, rr, vv, tau_dt) != 0);
  };
  double acc[3];
  kick_accel(table, np, mu, rrem, r, acc);
  int hit = within(table, np, rrem, r);
  if (hit >= 0) return {step0, ENCOUNTER, hit};
  if (escaped(r)) return {step0, ESCAPE, -1};
  *encounter_steps = 0;
  for (int64_t i = 0; i < nsteps; ++i) {
    const double* rowa = table + i * rowlen;
    const double* rowb = table + (i + 1) * rowlen;
    if (within(rowa, np, renc, r) < 0) {
      // the plain map step
      double rn[3], vn[3];
      for (int k = 0; k < 3; ++k) { rn[k] = r[k]; vn[k] = v[k] + 0.5 * dt * acc[k]; }
      if (!drift_or_fallback(rn, vn, dt)) return {step0 + i, KEPLER, -1};
      hit = kick_accel(rowb, np, mu, rrem, rn, acc);
      for (int k = 0; k < 3; ++k) { r[k] = rn[k]; v[k] = vn[k] + 0.5 * dt * acc[k]; }
      if (hit >= 0) return {step0 + i + 1, ENCOUNTER, hit};
    } else {
      // an encounter step of M substeps
      ++*encounter_steps;
      const double* va = vtable + i * 3 * np;
      const double* vb = vtable + (i + 1) * 3 * np;
      for (int m = 0; m < M; ++m) {
        double rn[3], vn[3];
        for (int k = 0; k < 3; ++k) { rn[k] = r[k]; vn[k] = v[k] + 0.5 * h * acc[k]; }
        if (!drift_or_fallback(rn, vn, h)) return {step0 + i, KEPLER, -1};
        if (m + 1 == M) {
          hit = kick_accel(rowb, np, mu, rrem, rn, acc);
        } else {
          hit = interp_accel((double)(m + 1) / M, dt, np, mu, rrem, rowa, va, rowb, vb, rn, acc);
        }
        for (int k = 0; k < 3; ++k) { r[k] = rn[k]; v[k] = vn[k] + 0.5 * h * acc[k]; }
        if (hit >= 0) return {step0 + i + 1, ENCOUNTER, hit};
      }
    }
    if (escaped(r)) return {step0 + i + 1, ESCAPE, -1};
  }
  return {-1, ACTIVE, -1};
}

// ---------------------------------------------------------------------------
// Osculating heliocentric elements of (r, v) about mu by the textbook
// two-body relations: a = 1/(2/r - v^2/mu); e from the eccentricity vector
// ((v^2 - mu/r) r - (r.v) v)/mu; h = r x v gives the inclination and the
// ascending node; the argument of latitude u (node to position, in the orbit
// plane); e cos E = 1 - r/a and e sin E = r.v / sqrt(mu a) give the eccentric
// anomaly E and the mean anomaly M = E - e sin E; the true anomaly f follows
// from E by f - E = 2 atan(beta sin E / (1 - beta cos E)), beta =
// e / (1 + sqrt(1 - e^2)), and the argument of pericentre is u - f.  Written
// this way the mean longitude node + (u - f) + M stays accurate on a circular
// orbit, where the pericentre itself is undefined.
// ---------------------------------------------------------------------------
struct Elements {
  double a, e, inc, node, peri, M;
};

Elements elements_of(double mu, const double* r, const double* v) {
  const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double rv = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
  Elements el;
  el.a = 1.0 / (2.0 / rn - v2 / mu);
  const double h[3] = {r[1] * v[2] - r[2] * v[1], r[2] * v[0] - r[0] * v[2],
                       r[0] * v[1] - r[1] * v[0]};
  double ev[3];
  for (int k = 0; k < 3; ++k) ev[k] = ((v2 - mu / rn) * r[k] - rv * v[k]) / mu;
  el.e = std::sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
  const double hn = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  el.inc = std::atan2(std::sqrt(h[0] * h[0] + h[1] * h[1]), h[2]);
  el.node = std::atan2(h[0], -h[1]);
  const double n[3] = {std::cos(el.node), std::sin(el.node), 0.0};
  // in the orbit plane, 90 degrees ahead of the node: (h/|h|) x n
  const double m[3] = {(h[1] * n[2] - h[2] * n[1]) / hn, (h[2] * n[0] - h[0] * n[2]) / hn,
                       (h[0] * n[1] - h[1] * n[0]) / hn};
  const double u = std::atan2(r[0] * m[0] + r[1] * m[1] + r[2] * m[2],
                              r[0] * n[0] + r[1] * n[1] + r[2] * n[2]);
  const double es = rv / std::sqrt(mu * el.a), ec = 1.0 - rn / el.a;
  const double E = std::atan2(es, ec);
  const double b = 1.0 + std::sqrt(1.0 - (ec * ec + es * es));
  const double f = E + 2.0 * std::atan2(es / b, 1.0 - ec / b);
  el.peri = u - f;
  el.M = E - es;
  return el;
}

// Mean longitude varpi + M (varpi = node + peri, the longitude of pericentre).
double mean_longitude(const Elements& el) { return el.node + el.peri + el.M; }

// ---------------------------------------------------------------------------
// Diagnostics of the paper's applications, sampled at every step boundary that
// is a multiple of `every` and that the particle reaches while active (the
// synchronised state (r_n, v_n), after that boundary's checks):
//  * the largest osculating eccentricity and the first sample that reached it
//    (sec. 3.3, maximum-eccentricity figure);
//  * for resonances (p, q) with a reference planet, the resonant angle
//      phi = p lambda - q lambda_ref - (p - q) varpi       (sec. 4.1),
//    with lambda the mean longitude and varpi the longitude of pericentre;
//    bit 0 of the flags records a sample with phi within 10 degrees of 0,
//    bit 1 one within 10 degrees of 180 degrees, so the paper's libration
//    criterion (sec. 4.2: phi never within 10 degrees of 0, or never within 10
//    degrees of 180) holds when the flags are not both set; lo and hi track
//    the range of phi - 180 degrees, taken in (-180, 180] degrees.
// ---------------------------------------------------------------------------
const double kTenDeg = M_PI / 18.0;

double wrap_angle(double x) { return std::remainder(x, kTwoPi); }

struct DiagSampler {
  double mu0;
  int64_t every;
  const double* lam_rows;      // lambda of the reference planet per table row (may be null)
  int nres;
  const int* p;
  const int* q;
  double* emax;
  int64_t* emax_step;
  int32_t* flags;
  double* lo;
  double* hi;
  double* margin;              // nearest approach of |phi| or |phi - 180 deg| to 10 degrees
  void operator()(int64_t n, int64_t row, const double* r, const double* v) const {
    if (n % every != 0) return;
    const Elements el = elements_of(mu0, r, v);
    if (el.e > *emax) {
      *emax = el.e;
      *emax_step = n;
    }
    if (!lam_rows) return;
    const double varpi = el.node + el.peri;
    const double lam = varpi + el.M;
    for (int k = 0; k < nres; ++k) {
      const double phi = p[k] * lam - q[k] * lam_rows[row] - (p[k] - q[k]) * varpi;
      const double w0 = wrap_angle(phi), w180 = wrap_angle(phi - M_PI);
      if (std::fabs(w0) < kTenDeg) flags[k] |= 1;
      if (std::fabs(w180) < kTenDeg) flags[k] |= 2;
      lo[k] = std::fmin(lo[k], w180);
      hi[k] = std::fmax(hi[k], w180);
      margin[k] = std::fmin(margin[k], std::fmin(std::fabs(std::fabs(w0) - kTenDeg),
                                                 std::fabs(std::fabs(w180) - kTenDeg)));
    }
  }
};

// ---------------------------------------------------------------------------
// Planet ephemeris: Wisdom-Holman map in Jacobi coordinates (sec. 2.2; Jacobi
// definitions as in sec. 2.2's coordinate list, with eta_i = sum_{j<=i} m_j).
// Bodies are 0 (central mass, heliocentric origin) and 1..np (sorted by a).
// ---------------------------------------------------------------------------
struct Planets {
  int np;
  double mu0;
  std::vector<double> mu;    // mu[0] = mu0, mu[j] = G m_j (j = 1..np)
  std::vector<double> eta;   // eta[j] = sum_{k<=j} mu[k]
  std::vector<double> rj, vj;  // Jacobi r', v' for j = 1..np at index 3(j-1)
  std::vector<double> a0;      // initial osculating semi-major axis (mu0 + mu_j), j = 1..np
};

// Heliocentric positions from Jacobi: r_j = r'_j + R_{j-1},
// R_j = (eta_{j-1} R_{j-1} + mu_j r_j) / eta_j, R_0 = 0.
void jacobi_to_helio(const Planets& P, const double* rj, double* rh) {
  double R[3] = {0, 0, 0};
  for (int j = 1; j <= P.np; ++j) {
    for (int k = 0; k < 3; ++k) rh[3 * (j - 1) + k] = rj[3 * (j - 1) + k] + R[k];
    for (int k = 0; k < 3; ++k)
      R[k] = (P.eta[j - 1] * R[k] + P.mu[j] * rh[3 * (j - 1) + k]) / P.eta[j];
  }
}

// Jacobi from heliocentric: r'_j = r_j - (sum_{k=1}^{j-1} mu_k r_k) / eta_{j-1}.
void helio_to_jacobi(const Planets& P, const double* rh, double* rj) {
  for (int j = 1; j <= P.np; ++j) {
    double S[3] = {0, 0, 0};
    for (int k = 1; k < j; ++k)
      for (int c = 0; c < 3; ++c) S[c] += P.mu[k] * rh[3 * (k - 1) + c];
    for (int c = 0; c < 3; ++c) rj[3 * (j - 1) + c] = rh[3 * (j - 1) + c] - S[c] / P.eta[j - 1];
  }
}

// Interaction acceleration of each Jacobi body (the kick part of the map):
//   a'_j = a_j - (sum_{k=0}^{j-1} mu_k a_k) / eta_{j-1} + mu'_j r'_j / |r'_j|^3,
// with a_k the full Newtonian acceleration of body k (body 0 at the origin) and
// mu'_j = mu0 eta_j / eta_{j-1} the Jacobi Kepler constant.
void jacobi_int_accel(const Planets& P, const double* rj, double* aj) {
  const int np = P.np;
  std::vector<double> pos(3 * (np + 1), 0.0), a(3 * (np + 1), 0.0);
  jacobi_to_helio(P, rj, pos.data() + 3);
  for (int k = 0; k <= np; ++k)
    for (int l = 0; l <= np; ++l) {
      if (l == k) continue;
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = pos[3 * k + c] - pos[3 * l + c];
      double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double d3 = d2 * std::sqrt(d2);
      for (int c = 0; c < 3; ++c) a[3 * k + c] -= P.mu[l] * d[c] / d3;
    }
  for (int j = 1; j <= np; ++j) {
    double S[3] = {0, 0, 0};
    for (int k = 0; k < j; ++k)
      for (int c = 0; c < 3; ++c) S[c] += P.mu[k] * a[3 * k + c];
    const double* r = rj + 3 * (j - 1);
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double r3 = r2 * std::sqrt(r2);
    double mup = P.mu0 * P.eta[j] / P.eta[j - 1];
    for (int c = 0; c < 3; ++c)
      aj[3 * (j - 1) + c] = a[3 * j + c] - S[c] / P.eta[j - 1] + mup * r[c] / r3;
  }
}

// Table row: heliocentric r_1..r_np and h0 = -sum_j mu_j r_j / |r_j|^3.
void write_row(const Planets& P, double* row) {
  jacobi_to_helio(P, P.rj.data(), row);
  double h0[3] = {0, 0, 0};
  for (int j = 1; j <= P.np; ++j) {
    const double* r = row + 3 * (j - 1);
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double r3 = r2 * std::sqrt(r2);
    for (int c = 0; c < 3; ++c) h0[c] -= P.mu[j] * r[c] / r3;
  }
  for (int c = 0; c < 3; ++c) row[3 * P.np + c] = h0[c];
}

// Any pair closer than one mutual Hill radius ((mu_i+mu_j)/(3 mu0))^(1/3) times
// the mean of their initial osculating semi-major axes.
bool planets_too_close(const Planets& P, const double* rh) {
  for (int i = 1; i <= P.np; ++i)
    for (int j = i + 1; j <= P.np; ++j) {
      const double* a = rh + 3 * (i - 1);
      const double* b = rh + 3 * (j - 1);
      double d2 = 0;
      for (int c = 0; c < 3; ++c) d2 += (a[c] - b[c]) * (a[c] - b[c]);
      double rh_m = std::cbrt((P.mu[i] + P.mu[j]) / (3.0 * P.mu0)) * 0.5 * (P.a0[i] + P.a0[j]);
      if (std::sqrt(d2) < rh_m) return true;
    }
  return false;
}

}  // namespace

extern "C" {

// ----------------------------- unit-level entry points ----------------------
double orc_kepler_solve(double ec, double es, double dM, int* iters) {
  return kep_solve<double>(ec, es, dM, iters);
}
double orc_kepler_fixedk(double ec, double es, double dM, int k, double* F) {
  double x = kep_fixedk<double>(ec, es, dM, k);
  if (F) *F = kep_F<double>(x, ec, es, dM);
  return x;
}
// Drift of a single two-body orbit (kfix < 0: no fixed-k decision).  fg[4] gets
// f, g, fdot, gdot when non-null.  Returns 1 on success, 0 on Kepler failure.
// Universal-variable drift of one state; returns 0 if it failed.
int orc_drift_universal(double mu, double* r, double* v, double dt) {
  return drift_universal(mu, r, v, dt);
}
int orc_drift(double mu, double* r, double* v, double dt, int kfix, double ftol, double* fg) {
  KepOut o{};
  int ok = drift<double>(mu, r, v, dt, kfix, ftol, &o);
  if (fg && ok) { fg[0] = o.f; fg[1] = o.g; fg[2] = o.fd; fg[3] = o.gd; }
  return ok;
}

// ----------------------------- planet ephemeris -----------------------------
// mu0; np planets with mu[np], heliocentric r[np*3], v[np*3] (sorted by a).
// Writes table[(nsteps+1) * (3np+3)] (row n = state at t_n), the final
// heliocentric r_out, v_out and, if vtable is not null, the heliocentric
// planet velocities vtable[(nsteps+1) * 3np].  Returns the first step at which two planets were
// within a mutual Hill radius, -2 if a planet's drift failed, else -1.
int64_t orc_ephemeris(double mu0, int np, const double* mu, const double* r, const double* v,
                      int64_t nsteps, double dt, double* table, double* r_out, double* v_out,
                      double* vtable) {
  Planets P;
  P.np = np;
  P.mu0 = mu0;
  P.mu.assign(np + 1, 0.0);
  P.eta.assign(np + 1, 0.0);
  P.mu[0] = mu0;
  P.eta[0] = mu0;
  for (int j = 1; j <= np; ++j) { P.mu[j] = mu[j - 1]; P.eta[j] = P.eta[j - 1] + P.mu[j]; }
  P.rj.assign(3 * np, 0.0);
  P.vj.assign(3 * np, 0.0);
  P.a0.assign(np + 1, 0.0);
  for (int j = 1; j <= np; ++j) {
    const double* rr = r + 3 * (j - 1);
    const double* vv = v + 3 * (j - 1);
    double rn = std::sqrt(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
    double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
    P.a0[j] = 1.0 / (2.0 / rn - v2 / (mu0 + P.mu[j]));
  }
  helio_to_jacobi(P, r, P.rj.data());
  helio_to_jacobi(P, v, P.vj.data());
  const int rowlen = 3 * np + 3;
  int64_t flag = -1;
  if (table) write_row(P, table);
  if (vtable) jacobi_to_helio(P, P.vj.data(), vtable);
  {
    std::vector<double> rh(3 * np);
    jacobi_to_helio(P, P.rj.data(), rh.data());
    if (np > 0 && planets_too_close(P, rh.data())) flag = 0;
  }
  std::vector<double> aj(3 * np), rh(3 * np);
  const double h = 0.5 * dt;
  for (int64_t s = 0; s < nsteps; ++s) {
    jacobi_int_accel(P, P.rj.data(), aj.data());
    for (int i = 0; i < 3 * np; ++i) P.vj[i] = P.vj[i] + h * aj[i];
    for (int j = 1; j <= np; ++j) {
      double mup = mu0 * P.eta[j] / P.eta[j - 1];
      if (!drift<double>(mup, &P.rj[3 * (j - 1)], &P.vj[3 * (j - 1)], dt, -1, 0.0) && flag == -1)
        flag = -2;
    }
    jacobi_int_accel(P, P.rj.data(), aj.data());
    for (int i = 0; i < 3 * np; ++i) P.vj[i] = P.vj[i] + h * aj[i];
    if (table) write_row(P, table + (s + 1) * rowlen);
    if (vtable) jacobi_to_helio(P, P.vj.data(), vtable + (s + 1) * 3 * np);
    jacobi_to_helio(P, P.rj.data(), rh.data());
    if (flag == -1 && np > 1 && planets_too_close(P, rh.data())) flag = s + 1;
  }
  if (r_out) jacobi_to_helio(P, P.rj.data(), r_out);
  if (v_out) jacobi_to_helio(P, P.vj.data(), v_out);
  return flag;
}

// ----------------------------- test particles -------------------------------
// Advances n particles (AoS r[n*3], v[n*3], in/out) through the table rows
// 0..nsteps (row 0 = global step step0).  Writes deact_step (-1 = survived),
// reason and planet (-1 if none).  With universal != 0 a drift the elliptic
// solve refuses is taken in universal variables instead of removing the
// particle.  Returns wall seconds of the particle loop.
double orc_particles(double mu0, int np, const double* mu, const double* rcrit, double rmax,
                     const double* table, int64_t nsteps, double dt, int64_t step0,
                     int kfix, double ftol, int64_t n, double* r, double* v,
                     int64_t* deact_step, int32_t* reason, int32_t* planet, int nthreads,
                     int universal) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  auto t0 = std::chrono::steady_clock::now();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    Deact d = run_particle<double>(mu0, np, mu, rcrit, rmax, table, nsteps, dt, step0, kfix,
                                   ftol, r + 3 * i, v + 3 * i, NoSample(), universal != 0);
    deact_step[i] = d.step;
    reason[i] = d.reason;
    planet[i] = d.planet;
  }
  auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count();
}

// Particles with the close-encounter hand-off (run_particle_handoff); the
// state arrays are updated in place; encounter_steps[n] (may be null).
double orc_particles_handoff(double mu0, int np, const double* mu, const double* renc,
                             const double* rrem, double rmax, const double* table,
                             const double* vtable, int64_t nsteps, double dt, int64_t step0,
                             int kfix, double ftol, int universal, int M, int64_t n, double* r,
                             double* v, int64_t* deact_step, int32_t* reason, int32_t* planet,
                             int64_t* encounter_steps, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  auto t0 = std::chrono::steady_clock::now();
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    int64_t es = 0;
    Deact d = run_particle_handoff(mu0, np, mu, renc, rrem, rmax, table, vtable, nsteps, dt, step0,
                                   kfix, ftol, universal != 0, M, r + 3 * i, v + 3 * i, &es);
    deact_step[i] = d.step;
    reason[i] = d.reason;
    planet[i] = d.planet;
    if (encounter_steps) encounter_steps[i] = es;
  }
  auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count();
}

// Planet table from a history of planet states (sec. 2.2: the planet
// positions shared by the particles may come from any source, such as
// interpolation from a history file).  Records k = 0..nrec-1 at strictly
// increasing times t[k] hold heliocentric positions hr[k][np][3] and
// velocities hv[k][np][3].  Row n of the table is the time t0 + n dt: each
// planet's position there is the cubic Hermite interpolant of the two records
// around it (the cubic matching both positions and both velocities), and h0 =
// -sum_j mu_j r_j / |r_j|^3 from those positions.  When vtable is not null it
// receives the interpolant's derivative (the velocities), [nsteps+1][np][3].
// Returns -1, or the first row whose time lies outside [t[0], t[nrec-1]]
// (that row and the rest are left unwritten).
int64_t orc_history_table(int np, const double* mu, int64_t nrec, const double* t,
                          const double* hr, const double* hv, double t0, double dt,
                          int64_t nsteps, double* table, double* vtable) {
  const int rowlen = 3 * np + 3;
  int64_t k = 0;
  for (int64_t n = 0; n <= nsteps; ++n) {
    const double tn = t0 + (double)n * dt;
    if (!(tn >= t[0] && tn <= t[nrec - 1])) return n;
    // the record interval [t[k], t[k+1]] containing tn (rows may run either way)
    while (k > 0 && tn < t[k]) --k;
    while (k + 1 < nrec - 1 && tn > t[k + 1]) ++k;
    const int64_t k1 = nrec > 1 ? k + 1 : k;
    const double h = t[k1] - t[k];
    const double s = h > 0.0 ? (tn - t[k]) / h : 0.0;
    // Hermite basis on [0, 1] and its derivative
    const double h00 = 2.0 * s * s * s - 3.0 * s * s + 1.0;
    const double h10 = s * s * s - 2.0 * s * s + s;
    const double h01 = -2.0 * s * s * s + 3.0 * s * s;
    const double h11 = s * s * s - s * s;
    const double d00 = 6.0 * s * s - 6.0 * s;
    const double d10 = 3.0 * s * s - 4.0 * s + 1.0;
    const double d01 = -6.0 * s * s + 6.0 * s;
    const double d11 = 3.0 * s * s - 2.0 * s;
    double* row = table + n * rowlen;
    double h0[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < np; ++j) {
      const double* pa = hr + (k * np + j) * 3;
      const double* pb = hr + (k1 * np + j) * 3;
      const double* va = hv + (k * np + j) * 3;
      const double* vb = hv + (k1 * np + j) * 3;
      for (int c = 0; c < 3; ++c) {
        row[3 * j + c] = h00 * pa[c] + h10 * h * va[c] + h01 * pb[c] + h11 * h * vb[c];
        if (vtable)
          vtable[(n * np + j) * 3 + c] =
              h > 0.0 ? (d00 * pa[c] + d01 * pb[c]) / h + d10 * va[c] + d11 * vb[c] : va[c];
      }
      const double* r = row + 3 * j;
      const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      const double r3 = r2 * std::sqrt(r2);
      for (int c = 0; c < 3; ++c) h0[c] -= mu[j] * r[c] / r3;
    }
    for (int c = 0; c < 3; ++c) row[3 * np + c] = h0[c];
  }
  return -1;
}

// Operations of one particle step of the method, per particle: the tally of
// run_particle over two steps less that over one (the steady state, in which
// the acceleration that ends a step also opens the next), for particles that
// stay active through both (Counted above says what is tallied).  out[5 i ..]
// = adds, multiplies, reciprocals, square roots, sine-cosine pairs; returns
// the number of particles counted (the others get -1).
int64_t orc_count_ops(double mu0, int np, const double* mu, const double* rcrit, double rmax,
                      const double* table, double dt, int kfix, double ftol, int64_t n,
                      const double* r, const double* v, int64_t* out) {
  int64_t counted = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t t[2][5];
    bool ok = true;
    for (int steps = 1; steps <= 2; ++steps) {
      Counted rc[3], vc[3];
      for (int k = 0; k < 3; ++k) { rc[k] = r[3 * i + k]; vc[k] = v[3 * i + k]; }
      g_tally = OpTally();
      g_tally.on = true;
      Deact d = run_particle<Counted>(mu0, np, mu, rcrit, rmax, table, steps, dt, 0, kfix, ftol,
                                      rc, vc);
      g_tally.on = false;
      ok = ok && d.reason == ACTIVE;
      t[steps - 1][0] = g_tally.add;
      t[steps - 1][1] = g_tally.mul;
      t[steps - 1][2] = g_tally.rcp;
      t[steps - 1][3] = g_tally.sqrt;
      t[steps - 1][4] = g_tally.sincos;
    }
    for (int k = 0; k < 5; ++k) out[5 * i + k] = ok ? t[1][k] - t[0][k] : -1;
    counted += ok ? 1 : 0;
  }
  return counted;
}

// orc_particles with the diagnostics above: every > 0; lam_rows[nsteps + 1]
// (mean longitude of the reference planet at each table row, read at sample
// rows; null for e_max only); nres <= 2 resonances p[k]:q[k].  Outputs per
// particle: emax (-1 without a sample), emax_step (-1), flags[n][nres],
// lo[n][nres], hi[n][nres] (radians; +inf / -inf without a sample).
double orc_particles_diag(double mu0, int np, const double* mu, const double* rcrit, double rmax,
                          const double* table, int64_t nsteps, double dt, int64_t step0, int kfix,
                          double ftol, int64_t n, double* r, double* v, int64_t* deact_step,
                          int32_t* reason, int32_t* planet, int nthreads, int64_t every,
                          const double* lam_rows, int nres, const int* p, const int* q,
                          double* emax, int64_t* emax_step, int32_t* flags, double* lo,
                          double* hi, double* margin) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  auto t0 = std::chrono::steady_clock::now();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    emax[i] = -1.0;
    emax_step[i] = -1;
    for (int k = 0; k < nres; ++k) {
      flags[nres * i + k] = 0;
      lo[nres * i + k] = INFINITY;
      hi[nres * i + k] = -INFINITY;
      margin[nres * i + k] = INFINITY;
    }
    DiagSampler smp{mu0, every, lam_rows, nres, p, q, emax + i, emax_step + i, flags + nres * i,
                    lo + nres * i, hi + nres * i, margin + nres * i};
    Deact d = run_particle<double>(mu0, np, mu, rcrit, rmax, table, nsteps, dt, step0, kfix,
                                   ftol, r + 3 * i, v + 3 * i, smp);
    deact_step[i] = d.step;
    reason[i] = d.reason;
    planet[i] = d.planet;
  }
  auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count();
}

// Osculating elements (a, e, inc, node, peri, M) of n states about mu: out[n][6].
void orc_elements(double mu, int64_t n, const double* r, const double* v, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const Elements el = elements_of(mu, r + 3 * i, v + 3 * i);
    const double e6[6] = {el.a, el.e, el.inc, el.node, el.peri, el.M};
    for (int k = 0; k < 6; ++k) out[6 * i + k] = e6[k];
  }
}

// Mean longitudes of n states about mu.
void orc_mean_longitudes(double mu, int64_t n, const double* r, const double* v, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = mean_longitude(elements_of(mu, r + 3 * i, v + 3 * i));
}

// Number of OpenMP threads a parallel region would use.
int orc_max_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

// Tangent of the particle map by the complex step: for each particle i the
// directional derivative of its final (r, v) along (dr[i], dv[i]) is written to
// dr_out, dv_out.  r, v are the initial states (not modified).  A particle
// deactivated at step n has the derivative of its frozen state (r_n, v_n).
void orc_tangent(double mu0, int np, const double* mu, const double* rcrit, double rmax,
                 const double* table, int64_t nsteps, double dt, int kfix, double ftol,
                 int64_t n, const double* r, const double* v, const double* dr, const double* dv,
                 double* dr_out, double* dv_out, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  const double hstep = 1e-100;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    cplx rc[3], vc[3];
    for (int k = 0; k < 3; ++k) {
      rc[k] = cplx(r[3 * i + k], hstep * dr[3 * i + k]);
      vc[k] = cplx(v[3 * i + k], hstep * dv[3 * i + k]);
    }
    run_particle<cplx>(mu0, np, mu, rcrit, rmax, table, nsteps, dt, 0, kfix, ftol, rc, vc);
    for (int k = 0; k < 3; ++k) {
      dr_out[3 * i + k] = rc[k].imag() / hstep;
      dv_out[3 * i + k] = vc[k].imag() / hstep;
    }
  }
}

}  // extern "C"
