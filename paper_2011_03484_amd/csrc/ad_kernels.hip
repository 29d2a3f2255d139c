// Tangent and adjoint kernels of the particle map (see ad.hpp for the math).
//
// Layout: particle states and adjoint/tangent vectors are structure-of-arrays
// blocks [6][n] (x, y, z, vx, vy, vz).  The planet table of the whole run is
// resident in HBM (row k = step k), so every segment can be recomputed.
//
//  * ad_segment   - steps [s0, s1) from a checkpoint; optionally writes a
//                   tape [s1-s0][AD_TAPE_FIELDS][n]: per step carried out,
//                   the state at its start, its opening acceleration and its
//                   Kepler root (x, sin x, cos x - 1).
//  * ad_reverse   - walks a segment's tape backwards applying the transposed
//                   step Jacobian to the adjoint vector kept in registers; the
//                   taped values spare it the Kepler solve and the opening
//                   acceleration, and give the same bits as recomputing them.
//  * ad_tangent   - carries (state, tangent) forward through [s0, s1).
#include "ad.hpp"
#include "ad_internal.h"

namespace tpm {

template <int NP>
struct ADArgs {
  PlanetConst<NP> P;
  KepConst K;
  double rmax2, ftol, dt;
  int kiters;
  int64_t n;
  int s0, s1;
};

template <int NP>
static ADArgs<NP> make_args(const SysConst& S, double dt, int64_t n, int s0, int s1) {
  ADArgs<NP> A;
  for (int j = 0; j < NP; ++j) { A.P.mu[j] = S.mu[j]; A.P.rcrit2[j] = S.rcrit2[j]; }
  if (NP == 0) { A.P.mu[0] = 0.0; A.P.rcrit2[0] = 0.0; }
  A.K = KepConst{S.mu0, S.inv_mu0, S.sqrt_mu0, S.inv_sqrt_mu0};
  A.rmax2 = S.rmax2;
  A.ftol = S.ftol;
  A.dt = dt;
  A.kiters = S.kiters;
  A.n = n;
  A.s0 = s0;
  A.s1 = s1;
  return A;
}

// One step of the map from (r, v) at step s (rows s, s+1), with the checks at
// its end.  Returns the new removal reason (ST_ACTIVE if none).
// row1: row s + 1 (a pointer, or a Row held in registers); xsm receives the
// drift's Kepler root, its sin and cos - 1.
template <int NP, typename RowT>
TPM_DEV int32_t ad_step(const ADArgs<NP>& A, const RowT& row1, double r[3], double v[3],
                        double acc[3], int32_t& planet, double xsm[3]) {
  const double h = 0.5 * A.dt;
  DriftVals D;
  double nr[3], nv[3];
  drift_vals(A.K, A.dt, A.kiters, A.ftol, r[0], r[1], r[2], fma_(h, acc[0], v[0]),
             fma_(h, acc[1], v[1]), fma_(h, acc[2], v[2]), D, nr[0], nr[1], nr[2], nv[0], nv[1],
             nv[2]);
  xsm[0] = D.x; xsm[1] = D.s; xsm[2] = D.m;
  if (!D.ok) return ST_KEPLER;
  double b[3];
  int hit = accel<NP>(row1, A.P, nr[0], nr[1], nr[2], b[0], b[1], b[2]);
  for (int k = 0; k < 3; ++k) {
    r[k] = nr[k];
    acc[k] = b[k];
    v[k] = fma_(h, b[k], nv[k]);
  }
  if (hit >= 0) { planet = hit; return ST_ENCOUNTER; }
  if (fma_(r[0], r[0], fma_(r[1], r[1], r[2] * r[2])) > A.rmax2) return ST_ESCAPE;
  return ST_ACTIVE;
}

// mode 0: first segment (removal records initialised, checks at step s0);
// mode 1: later segment (records read and updated);
// mode 2: recompute for the adjoint - a particle advances exactly through the
//         steps s < dstep[i] of the recorded run and no record is written.
template <int NP>
__global__ void __launch_bounds__(256)
ad_segment(ADArgs<NP> A, const double* __restrict__ table, const double* __restrict__ in,
           double* __restrict__ out, double* __restrict__ tape, int64_t* __restrict__ dstep,
           int32_t* __restrict__ reason, int32_t* __restrict__ planet, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  constexpr int ROW = 3 * NP + 3;
  const int64_t n = A.n;
  double r[3] = {in[i], in[n + i], in[2 * n + i]};
  double v[3] = {in[3 * n + i], in[4 * n + i], in[5 * n + i]};
  int32_t why = ST_ACTIVE, pl = -1;
  int64_t ds = -1;
  if (mode == 1) { why = reason[i]; pl = planet[i]; ds = dstep[i]; }
  // last step (exclusive) to carry out in recompute mode
  int64_t stop = A.s1;
  if (mode == 2) {
    const int64_t d = dstep[i];
    if (d >= 0 && d < stop) stop = d;
  }
  double acc[3];
  int hit = accel<NP>(table + (size_t)A.s0 * ROW, A.P, r[0], r[1], r[2], acc[0], acc[1], acc[2]);
  if (mode == 0) {
    if (hit >= 0) { why = ST_ENCOUNTER; pl = hit; ds = A.s0; }
    else if (fma_(r[0], r[0], fma_(r[1], r[1], r[2] * r[2])) > A.rmax2) { why = ST_ESCAPE; ds = A.s0; }
  }
  // the row that ends step s is fetched into registers during step s - 1
  const int zero = opaque_zero_vgpr();
  Row<NP> R1, Rn;
  if (A.s0 < A.s1) load_row<NP>(R1, table + (size_t)(A.s0 + 1) * ROW, zero);
  for (int s = A.s0; s < A.s1; ++s) {
    if (s + 1 < A.s1) load_row<NP>(Rn, table + (size_t)(s + 2) * ROW, zero);
    const Row<NP> Rs = R1;
    R1 = Rn;
    if (mode == 2 ? (s >= stop) : (why != ST_ACTIVE)) continue;
    double r1[3] = {r[0], r[1], r[2]}, v1[3] = {v[0], v[1], v[2]}, a1[3] = {acc[0], acc[1], acc[2]};
    int32_t p1 = -1;
    double xsm[3];
    int32_t w = ad_step<NP>(A, Rs.v, r1, v1, a1, p1, xsm);
    if (w == ST_KEPLER) { why = w; ds = s; continue; }
    if (tape) {
      double* t = tape + (size_t)(s - A.s0) * AD_TAPE_FIELDS * n + i;
      const double f[AD_TAPE_FIELDS] = {r[0], r[1], r[2], v[0], v[1], v[2], acc[0], acc[1], acc[2],
                                        xsm[0], xsm[1], xsm[2]};
#pragma unroll
      for (int k = 0; k < AD_TAPE_FIELDS; ++k) t[(size_t)k * n] = f[k];
    }
    for (int k = 0; k < 3; ++k) { r[k] = r1[k]; v[k] = v1[k]; acc[k] = a1[k]; }
    if (w != ST_ACTIVE) { why = w; pl = p1; ds = s + 1; }
  }
  if (out) {
    out[i] = r[0]; out[n + i] = r[1]; out[2 * n + i] = r[2];
    out[3 * n + i] = v[0]; out[4 * n + i] = v[1]; out[5 * n + i] = v[2];
  }
  if (mode != 2) {
    reason[i] = why;
    planet[i] = pl;
    dstep[i] = ds;
  }
}

template <int NP>
__global__ void __launch_bounds__(256)
ad_reverse(ADArgs<NP> A, const double* __restrict__ table, const double* __restrict__ tape,
           double* __restrict__ lam, const int64_t* __restrict__ dstep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  constexpr int ROW = 3 * NP + 3;
  const int64_t n = A.n;
  const double h = 0.5 * A.dt;
  double lr[3] = {lam[i], lam[n + i], lam[2 * n + i]};
  double lv[3] = {lam[3 * n + i], lam[4 * n + i], lam[5 * n + i]};
  const int64_t ds = dstep[i];
  // steps s with s < ds (or all steps if never removed) were carried out
  int s_top = A.s1;
  if (ds >= 0 && ds < (int64_t)s_top) s_top = (int)(ds > A.s0 ? ds : A.s0);
  // the tape entry of step s is fetched during step s + 1 (its loads do not
  // depend on the adjoint)
  auto fetch = [&](int s, double (&f)[AD_TAPE_FIELDS]) {
    const double* t = tape + (size_t)(s - A.s0) * AD_TAPE_FIELDS * n + i;
#pragma unroll
    for (int k = 0; k < AD_TAPE_FIELDS; ++k) f[k] = t[(size_t)k * n];
  };
  // and so is row s - 1 (rows s and s + 1 are in registers already)
  double cur[AD_TAPE_FIELDS], nxt[AD_TAPE_FIELDS];
  Row<NP> R0, R1, Rn;
  if (s_top - 1 >= A.s0) {
    fetch(s_top - 1, cur);
    load_row<NP>(R0, table + (size_t)(s_top - 1) * ROW, 0);
    load_row<NP>(R1, table + (size_t)s_top * ROW, 0);
  }
  for (int s = s_top - 1; s >= A.s0; --s) {
    if (s - 1 >= A.s0) {
      fetch(s - 1, nxt);
      load_row<NP>(Rn, table + (size_t)(s - 1) * ROW, 0);
    }
    double r[3] = {cur[0], cur[1], cur[2]};
    double v[3] = {cur[3], cur[4], cur[5]};
    const auto& row0 = R0.v;
    const auto& row1 = R1.v;
    double vh[3] = {fma_(h, cur[6], v[0]), fma_(h, cur[7], v[1]), fma_(h, cur[8], v[2])};
    DriftVals D;
    double nr[3], nv[3];
    drift_vals_t<true>(A.K, A.dt, A.kiters, A.ftol, r[0], r[1], r[2], vh[0], vh[1], vh[2], D, nr[0],
                       nr[1], nr[2], nv[0], nv[1], nv[2], cur[9], cur[10], cur[11]);
    // closing kick: v_{s+1} = v' + h a(r_{s+1})
    double Al[3];
    accel_jac<NP>(row1, A.P, nr, lv, Al);
    double lr1[3] = {lr[0] + h * Al[0], lr[1] + h * Al[1], lr[2] + h * Al[2]};
    // drift
    double lr0[3], lvh[3];
    drift_vjp(A.K, A.dt, D, r, vh, lr1, lv, lr0, lvh);
    // opening kick: vh = v_s + h a(r_s)
    accel_jac<NP>(row0, A.P, r, lvh, Al);
    for (int k = 0; k < 3; ++k) {
      lr[k] = lr0[k] + h * Al[k];
      lv[k] = lvh[k];
    }
#pragma unroll
    for (int k = 0; k < AD_TAPE_FIELDS; ++k) cur[k] = nxt[k];
    R1 = R0;
    R0 = Rn;
  }
  lam[i] = lr[0]; lam[n + i] = lr[1]; lam[2 * n + i] = lr[2];
  lam[3 * n + i] = lv[0]; lam[4 * n + i] = lv[1]; lam[5 * n + i] = lv[2];
}

template <int NP>
__global__ void __launch_bounds__(256)
ad_tangent(ADArgs<NP> A, const double* __restrict__ table, double* __restrict__ st,
           double* __restrict__ tg, int32_t* __restrict__ reason, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  constexpr int ROW = 3 * NP + 3;
  const int64_t n = A.n;
  const double h = 0.5 * A.dt;
  double r[3] = {st[i], st[n + i], st[2 * n + i]};
  double v[3] = {st[3 * n + i], st[4 * n + i], st[5 * n + i]};
  double dr[3] = {tg[i], tg[n + i], tg[2 * n + i]};
  double dv[3] = {tg[3 * n + i], tg[4 * n + i], tg[5 * n + i]};
  int32_t why = first ? ST_ACTIVE : reason[i];
  double acc[3];
  int hit = accel<NP>(table + (size_t)A.s0 * ROW, A.P, r[0], r[1], r[2], acc[0], acc[1], acc[2]);
  if (first && (hit >= 0 || fma_(r[0], r[0], fma_(r[1], r[1], r[2] * r[2])) > A.rmax2))
    why = hit >= 0 ? ST_ENCOUNTER : ST_ESCAPE;
  for (int s = A.s0; s < A.s1 && why == ST_ACTIVE; ++s) {
    const double* row1 = table + (size_t)(s + 1) * ROW;
    double Ad[3];
    accel_jac<NP>(table + (size_t)s * ROW, A.P, r, dr, Ad);
    double vh[3] = {fma_(h, acc[0], v[0]), fma_(h, acc[1], v[1]), fma_(h, acc[2], v[2])};
    double dvh[3] = {dv[0] + h * Ad[0], dv[1] + h * Ad[1], dv[2] + h * Ad[2]};
    DriftVals D;
    double nr[3], nv[3];
    drift_vals(A.K, A.dt, A.kiters, A.ftol, r[0], r[1], r[2], vh[0], vh[1], vh[2], D, nr[0], nr[1],
               nr[2], nv[0], nv[1], nv[2]);
    if (!D.ok) { why = ST_KEPLER; break; }
    double ndr[3], ndv[3];
    drift_jvp(A.K, A.dt, D, r, vh, dr, dvh, ndr, ndv);
    double b[3];
    int h1 = accel<NP>(row1, A.P, nr[0], nr[1], nr[2], b[0], b[1], b[2]);
    accel_jac<NP>(row1, A.P, nr, ndr, Ad);
    for (int k = 0; k < 3; ++k) {
      r[k] = nr[k];
      acc[k] = b[k];
      v[k] = fma_(h, b[k], nv[k]);
      dr[k] = ndr[k];
      dv[k] = ndv[k] + h * Ad[k];
    }
    if (h1 >= 0) why = ST_ENCOUNTER;
    else if (fma_(r[0], r[0], fma_(r[1], r[1], r[2] * r[2])) > A.rmax2) why = ST_ESCAPE;
  }
  st[i] = r[0]; st[n + i] = r[1]; st[2 * n + i] = r[2];
  st[3 * n + i] = v[0]; st[4 * n + i] = v[1]; st[5 * n + i] = v[2];
  tg[i] = dr[0]; tg[n + i] = dr[1]; tg[2 * n + i] = dr[2];
  tg[3 * n + i] = dv[0]; tg[4 * n + i] = dv[1]; tg[5 * n + i] = dv[2];
  reason[i] = why;
}

// [n][3] r and v  <->  [6][n]
__global__ void __launch_bounds__(256)
aos_to_soa(const double* __restrict__ r, const double* __restrict__ v, double* __restrict__ o,
           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    o[k * n + i] = r[3 * i + k];
    o[(3 + k) * n + i] = v[3 * i + k];
  }
}

__global__ void __launch_bounds__(256)
soa_to_aos(const double* __restrict__ o, double* __restrict__ r, double* __restrict__ v,
           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    if (r) r[3 * i + k] = o[k * n + i];
    if (v) v[3 * i + k] = o[(3 + k) * n + i];
  }
}

static int grid_of(int64_t n) { return (int)((n + 255) / 256); }

// The derivative kernels run one particle per lane for a whole segment, and
// the derivative workloads are small (16,384 particles: 256 wavefronts for
// 1,024 SIMDs): one wavefront per workgroup spreads them over every compute
// unit instead of packing four onto each of 64.
constexpr int AD_BLOCK = 64;
static int ad_grid(int64_t n) { return (int)((n + AD_BLOCK - 1) / AD_BLOCK); }

hipError_t launch_aos_to_soa(const double* r, const double* v, double* o, int64_t n,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(aos_to_soa, dim3(grid_of(n)), dim3(256), 0, st, r, v, o, n);
  return hipGetLastError();
}

hipError_t launch_soa_to_aos(const double* o, double* r, double* v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(soa_to_aos, dim3(grid_of(n)), dim3(256), 0, st, o, r, v, n);
  return hipGetLastError();
}

#define TPM_NP_SWITCH(NPV, CALL) \
  switch (NPV) {                 \
    case 0: CALL(0); break;      \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    case 7: CALL(7); break;      \
    case 8: CALL(8); break;      \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_ad_segment(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, const double* in, double* out, double* tape,
                             int64_t* dstep, int32_t* reason, int32_t* planet, int mode,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
#define TPM_SEG(N)                                                                          \
  hipLaunchKernelGGL(ad_segment<N>, dim3(ad_grid(n)), dim3(AD_BLOCK), 0, st,                     \
                     make_args<N>(S, dt, n, s0, s1), table, in, out, tape, dstep, reason,   \
                     planet, mode)
  TPM_NP_SWITCH(S.np, TPM_SEG)
#undef TPM_SEG
  return hipGetLastError();
}

hipError_t launch_ad_reverse(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, const double* tape, double* lam,
                             const int64_t* dstep, hipStream_t st) {
  if (n <= 0) return hipSuccess;
#define TPM_REV(N)                                                                     \
  hipLaunchKernelGGL(ad_reverse<N>, dim3(ad_grid(n)), dim3(AD_BLOCK), 0, st,                \
                     make_args<N>(S, dt, n, s0, s1), table, tape, lam, dstep)
  TPM_NP_SWITCH(S.np, TPM_REV)
#undef TPM_REV
  return hipGetLastError();
}

hipError_t launch_ad_tangent(const SysConst& S, double dt, int64_t n, int s0, int s1,
                             const double* table, double* st_, double* tg, int32_t* reason,
                             bool first, hipStream_t st) {
  if (n <= 0) return hipSuccess;
#define TPM_TAN(N)                                                                     \
  hipLaunchKernelGGL(ad_tangent<N>, dim3(ad_grid(n)), dim3(AD_BLOCK), 0, st,                \
                     make_args<N>(S, dt, n, s0, s1), table, st_, tg, reason, first ? 1 : 0)
  TPM_NP_SWITCH(S.np, TPM_TAN)
#undef TPM_TAN
  return hipGetLastError();
}

}  // namespace tpm
