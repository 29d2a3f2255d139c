// Core kernels of the test-particle map on gfx950 (FP64 throughout).
//
//  * particle_chunk  - one lane per particle; the particle stays in registers
//    for a whole chunk of steps (sec. 2.2: a single kernel loops over the
//    planet chunk so each particle is read and written once per chunk).  Every
//    lane reads the same planet-table row, so the row is fetched with scalar
//    loads (wave-uniform address) into SGPRs.
//  * ephemeris_chunk - one wavefront; lane b holds Jacobi body b.  Wisdom-Holman
//    kick-drift-kick of the planets (sec. 2.2, planet integration) writing the
//    heliocentric positions and the indirect term h0 per step.
//  * compact_*       - stable partition of the working set so removed particles
//    stop occupying lanes (sec. 2.2, resync interval), by wave ballots, an LDS
//    scan and ordered block offsets.
//  * finalize        - scatter the active particles back to caller order.
#include "internal.h"
#include "particle.hpp"

namespace tpm {

// ---------------------------------------------------------------- particles
template <int NP>
struct ChunkArgs {
  PlanetConst<NP> P;
  KepConst K;
  double rmax2, ftol, dt;
  int kiters, nsteps;
  int64_t step0;
};

// KIT > 0 fixes the Newton count at compile time (fully unrolled); KIT == 0
// reads it from the arguments.
template <int NP, int KIT>
__global__ void __launch_bounds__(256)
particle_chunk(Work w, const int32_t* __restrict__ d_nactive, Out out,
               const double* __restrict__ rows, ChunkArgs<NP> A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_nactive) return;
  if (w.status[i] != ST_ACTIVE) return;
  constexpr int ROW = 3 * NP + 3;
  const int kiters = KIT > 0 ? KIT : A.kiters;
  double x = w.x[i], y = w.y[i], z = w.z[i];
  double vx = w.vx[i], vy = w.vy[i], vz = w.vz[i];
  double ax, ay, az;
  int hit = accel<NP>(rows, A.P, x, y, z, ax, ay, az);
  int32_t reason = ST_ACTIVE, planet = -1;
  int64_t dstep = -1;
  if (hit >= 0) {
    reason = ST_ENCOUNTER; planet = hit; dstep = A.step0;
  } else if (fma_(x, x, fma_(y, y, z * z)) > A.rmax2) {
    reason = ST_ESCAPE; dstep = A.step0;
  }
  const double h = 0.5 * A.dt;
  // The step loop is uniform across the wavefront (so the row address stays
  // wave-uniform and is read by scalar loads); removed lanes are masked off
  // and the wavefront leaves early once none of its lanes is active.
  for (int s = 0; s < A.nsteps; ++s) {
    if (__all(reason != ST_ACTIVE)) break;
    const double* row = rows + (size_t)(s + 1) * ROW;
    if (reason == ST_ACTIVE) {
      double nx = x, ny = y, nz = z;
      double nvx = fma_(h, ax, vx), nvy = fma_(h, ay, vy), nvz = fma_(h, az, vz);
      bool ok = drift_fixed(A.K, A.dt, kiters, A.ftol, nx, ny, nz, nvx, nvy, nvz);
      double bx, by, bz;
      int hit1 = accel<NP>(row, A.P, nx, ny, nz, bx, by, bz);
      double r2 = fma_(nx, nx, fma_(ny, ny, nz * nz));
      if (!ok) {
        reason = ST_KEPLER; dstep = A.step0 + s;
      } else {
        x = nx; y = ny; z = nz;
        ax = bx; ay = by; az = bz;
        vx = fma_(h, ax, nvx); vy = fma_(h, ay, nvy); vz = fma_(h, az, nvz);
        if (hit1 >= 0) {
          reason = ST_ENCOUNTER; planet = hit1; dstep = A.step0 + s + 1;
        } else if (r2 > A.rmax2) {
          reason = ST_ESCAPE; dstep = A.step0 + s + 1;
        }
      }
    }
  }
  if (reason != ST_ACTIVE) {
    const int k = w.slot[i];
    out.r[3 * k + 0] = x; out.r[3 * k + 1] = y; out.r[3 * k + 2] = z;
    out.v[3 * k + 0] = vx; out.v[3 * k + 1] = vy; out.v[3 * k + 2] = vz;
    out.step[k] = dstep;
    out.reason[k] = reason;
    out.planet[k] = planet;
    w.status[i] = reason;
  } else {
    w.x[i] = x; w.y[i] = y; w.z[i] = z;
    w.vx[i] = vx; w.vy[i] = vy; w.vz[i] = vz;
  }
}

template <int NP>
static hipError_t launch_np(const SysConst& S, Work w, const int32_t* d_nactive, int grid_n,
                            Out out, const double* rows, int nsteps, double dt, int64_t step0,
                            int block, hipStream_t st) {
  ChunkArgs<NP> A;
  for (int j = 0; j < NP; ++j) { A.P.mu[j] = S.mu[j]; A.P.rcrit2[j] = S.rcrit2[j]; }
  if (NP == 0) { A.P.mu[0] = 0.0; A.P.rcrit2[0] = 0.0; }
  A.K = KepConst{S.mu0, S.inv_mu0, S.sqrt_mu0, S.inv_sqrt_mu0};
  A.rmax2 = S.rmax2;
  A.ftol = S.ftol;
  A.dt = dt;
  A.kiters = S.kiters;
  A.nsteps = nsteps;
  A.step0 = step0;
  int grid = (grid_n + block - 1) / block;
  if (grid <= 0) return hipSuccess;
  if (S.kiters == 5)
    hipLaunchKernelGGL((particle_chunk<NP, 5>), dim3(grid), dim3(block), 0, st, w, d_nactive, out, rows, A);
  else
    hipLaunchKernelGGL((particle_chunk<NP, 0>), dim3(grid), dim3(block), 0, st, w, d_nactive, out, rows, A);
  return hipGetLastError();
}

hipError_t launch_particle_chunk(const SysConst& S, Work w, const int32_t* d_nactive, int grid_n,
                                 Out out, const double* rows, int nsteps, double dt, int64_t step0,
                                 int block, hipStream_t st) {
  switch (S.np) {
    case 0: return launch_np<0>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 1: return launch_np<1>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 2: return launch_np<2>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 3: return launch_np<3>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 4: return launch_np<4>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 5: return launch_np<5>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 6: return launch_np<6>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 7: return launch_np<7>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    case 8: return launch_np<8>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, block, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- ephemeris
// Value of v held by lane src (wave64 cross-lane read).
TPM_DEV double lane_read(double v, int src) { return __shfl(v, src, 64); }

// Heliocentric positions of bodies 1..NP from the Jacobi positions held by
// lanes 1..NP: r_b = r'_b + R_{b-1}, R_b = (eta_{b-1} R_{b-1} + mu_b r_b)/eta_b.
// Every lane computes the whole chain and keeps all positions.
template <int NP>
TPM_DEV void helio_all(const EphConst& E, double jx, double jy, double jz,
                       double (&hx)[NP + 1], double (&hy)[NP + 1], double (&hz)[NP + 1]) {
  double Rx = 0.0, Ry = 0.0, Rz = 0.0;
  hx[0] = 0.0; hy[0] = 0.0; hz[0] = 0.0;
#pragma unroll
  for (int b = 1; b <= NP; ++b) {
    double px = lane_read(jx, b) + Rx;
    double py = lane_read(jy, b) + Ry;
    double pz = lane_read(jz, b) + Rz;
    hx[b] = px; hy[b] = py; hz[b] = pz;
    // (eta_{b-1} R + mu_b r_b) / eta_b
    Rx = fma_(E.eta[b - 1], Rx, E.mu[b] * px) * E.inv_eta[b];
    Ry = fma_(E.eta[b - 1], Ry, E.mu[b] * py) * E.inv_eta[b];
    Rz = fma_(E.eta[b - 1], Rz, E.mu[b] * pz) * E.inv_eta[b];
  }
}

// Interaction acceleration of Jacobi body `lane` (lanes 1..NP) and, on lane 0,
// the central body's acceleration a_0 (h0 = -a_0).
//   a'_b = a_b - (sum_{k<b} mu_k a_k)/eta_{b-1} + mu'_b r'_b/|r'_b|^3
template <int NP>
TPM_DEV void eph_accel(const EphConst& E, int lane, double jx, double jy, double jz,
                       const double (&hx)[NP + 1], const double (&hy)[NP + 1],
                       const double (&hz)[NP + 1], double& ax, double& ay, double& az) {
  // own heliocentric position
  double ox = 0.0, oy = 0.0, oz = 0.0;
#pragma unroll
  for (int b = 0; b <= NP; ++b)
    if (lane == b) { ox = hx[b]; oy = hy[b]; oz = hz[b]; }
  // Newtonian acceleration of body `lane`
  double nx = 0.0, ny = 0.0, nz = 0.0;
#pragma unroll
  for (int l = 0; l <= NP; ++l) {
    double dx = ox - hx[l], dy = oy - hy[l], dz = oz - hz[l];
    double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
    bool self = (l == lane);
    double inv = rsqrt(self ? 1.0 : d2);
    double k = self ? 0.0 : E.mu[l] * (inv * inv) * inv;
    nx = fma_(-k, dx, nx);
    ny = fma_(-k, dy, ny);
    nz = fma_(-k, dz, nz);
  }
  // S = sum_{k<lane} mu_k a_k
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double kx = lane_read(nx, k), ky = lane_read(ny, k), kz = lane_read(nz, k);
    if (k < lane) {
      sx = fma_(E.mu[k], kx, sx);
      sy = fma_(E.mu[k], ky, sy);
      sz = fma_(E.mu[k], kz, sz);
    }
  }
  if (lane >= 1 && lane <= NP) {
    double ie = 0.0, mup = 0.0;
#pragma unroll
    for (int b = 1; b <= NP; ++b)
      if (lane == b) { ie = E.inv_eta[b - 1]; mup = E.mup[b]; }
    double r2 = fma_(jx, jx, fma_(jy, jy, jz * jz));
    double inv = rsqrt(r2);
    double k = mup * (inv * inv) * inv;
    ax = fma_(k, jx, fma_(-sx, ie, nx));
    ay = fma_(k, jy, fma_(-sy, ie, ny));
    az = fma_(k, jz, fma_(-sz, ie, nz));
  } else {
    ax = nx; ay = ny; az = nz;
  }
}

template <int NP>
TPM_DEV bool hill_violation(const EphConst& E, int lane, const double (&hx)[NP + 1],
                            const double (&hy)[NP + 1], const double (&hz)[NP + 1]) {
  bool bad = false;
#pragma unroll
  for (int i = 1; i <= NP; ++i)
#pragma unroll
    for (int j = i + 1; j <= NP; ++j) {
      if (lane != i) continue;
      double dx = hx[i] - hx[j], dy = hy[i] - hy[j], dz = hz[i] - hz[j];
      double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
      double ri = rsqrt(fma_(hx[i], hx[i], fma_(hy[i], hy[i], hz[i] * hz[i])));
      double rj = rsqrt(fma_(hx[j], hx[j], fma_(hy[j], hy[j], hz[j] * hz[j])));
      double ri_ = fma_(hx[i], hx[i], fma_(hy[i], hy[i], hz[i] * hz[i])) * ri;
      double rj_ = fma_(hx[j], hx[j], fma_(hy[j], hy[j], hz[j] * hz[j])) * rj;
      double lim = E.hill[i][j] * (ri_ + rj_);
      bad = bad || (d2 < lim * lim);
    }
  return bad;
}

template <int NP>
__global__ void __launch_bounds__(64)
ephemeris_chunk(EphConst E, double* __restrict__ rj, double* __restrict__ vj,
                double* __restrict__ rows, int nsteps, double dt, int64_t step0,
                int64_t* __restrict__ flag) {
  constexpr int ROW = 3 * NP + 3;
  const int lane = threadIdx.x;
  const bool body = lane >= 1 && lane <= NP;
  double jx = 0, jy = 0, jz = 0, wx = 0, wy = 0, wz = 0;
  if (body) {
    jx = rj[3 * (lane - 1) + 0]; jy = rj[3 * (lane - 1) + 1]; jz = rj[3 * (lane - 1) + 2];
    wx = vj[3 * (lane - 1) + 0]; wy = vj[3 * (lane - 1) + 1]; wz = vj[3 * (lane - 1) + 2];
  }
  double mup = 0.0;
#pragma unroll
  for (int b = 1; b <= NP; ++b)
    if (lane == b) mup = E.mup[b];
  double hx[NP + 1], hy[NP + 1], hz[NP + 1];
  double ax, ay, az;
  helio_all<NP>(E, jx, jy, jz, hx, hy, hz);
  eph_accel<NP>(E, lane, jx, jy, jz, hx, hy, hz, ax, ay, az);
  // row 0: current state
  if (body) {
    rows[3 * (lane - 1) + 0] = hx[lane];
    rows[3 * (lane - 1) + 1] = hy[lane];
    rows[3 * (lane - 1) + 2] = hz[lane];
  } else if (lane == 0) {
    rows[3 * NP + 0] = -ax; rows[3 * NP + 1] = -ay; rows[3 * NP + 2] = -az;
  }
  const double h = 0.5 * dt;
  int64_t bad_step = -1;
  for (int s = 0; s < nsteps; ++s) {
    wx = fma_(h, ax, wx); wy = fma_(h, ay, wy); wz = fma_(h, az, wz);
    bool bound = drift_converged(body ? mup : 1.0, dt, body, jx, jy, jz, wx, wy, wz);
    if (bad_step == -1 && __any(body && !bound)) bad_step = -2;
    helio_all<NP>(E, jx, jy, jz, hx, hy, hz);
    eph_accel<NP>(E, lane, jx, jy, jz, hx, hy, hz, ax, ay, az);
    wx = fma_(h, ax, wx); wy = fma_(h, ay, wy); wz = fma_(h, az, wz);
    double* row = rows + (size_t)(s + 1) * ROW;
    if (body) {
      row[3 * (lane - 1) + 0] = hx[lane];
      row[3 * (lane - 1) + 1] = hy[lane];
      row[3 * (lane - 1) + 2] = hz[lane];
    } else if (lane == 0) {
      row[3 * NP + 0] = -ax; row[3 * NP + 1] = -ay; row[3 * NP + 2] = -az;
    }
    if (bad_step == -1 && NP > 1 && __any(hill_violation<NP>(E, lane, hx, hy, hz)))
      bad_step = step0 + s + 1;
  }
  if (body) {
    rj[3 * (lane - 1) + 0] = jx; rj[3 * (lane - 1) + 1] = jy; rj[3 * (lane - 1) + 2] = jz;
    vj[3 * (lane - 1) + 0] = wx; vj[3 * (lane - 1) + 1] = wy; vj[3 * (lane - 1) + 2] = wz;
  }
  if (lane == 0 && bad_step != -1 && *flag == -1) *flag = bad_step;
}

template <int NP>
static hipError_t eph_np(const EphConst& E, double* rj, double* vj, double* rows, int nsteps,
                         double dt, int64_t step0, int64_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(ephemeris_chunk<NP>, dim3(1), dim3(64), 0, st, E, rj, vj, rows, nsteps, dt,
                     step0, flag);
  return hipGetLastError();
}

hipError_t launch_ephemeris_chunk(const EphConst& E, double* rj, double* vj, double* rows,
                                  int nsteps, double dt, int64_t step0, int64_t* flag,
                                  hipStream_t st) {
  switch (E.np) {
    case 0: return eph_np<0>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 1: return eph_np<1>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 2: return eph_np<2>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 3: return eph_np<3>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 4: return eph_np<4>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 5: return eph_np<5>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 6: return eph_np<6>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 7: return eph_np<7>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    case 8: return eph_np<8>(E, rj, vj, rows, nsteps, dt, step0, flag, st);
    default: return hipErrorInvalidValue;
  }
}

// Jacobi -> heliocentric positions and velocities of the planets (one wave).
template <int NP>
__global__ void __launch_bounds__(64)
jacobi_to_helio_kernel(EphConst E, const double* rj, const double* vj, double* rh, double* vh) {
  const int lane = threadIdx.x;
  const bool body = lane >= 1 && lane <= NP;
  double jx = 0, jy = 0, jz = 0, wx = 0, wy = 0, wz = 0;
  if (body) {
    jx = rj[3 * (lane - 1) + 0]; jy = rj[3 * (lane - 1) + 1]; jz = rj[3 * (lane - 1) + 2];
    wx = vj[3 * (lane - 1) + 0]; wy = vj[3 * (lane - 1) + 1]; wz = vj[3 * (lane - 1) + 2];
  }
  double hx[NP + 1], hy[NP + 1], hz[NP + 1];
  helio_all<NP>(E, jx, jy, jz, hx, hy, hz);
  double ux[NP + 1], uy[NP + 1], uz[NP + 1];
  helio_all<NP>(E, wx, wy, wz, ux, uy, uz);
  if (body) {
    rh[3 * (lane - 1) + 0] = hx[lane]; rh[3 * (lane - 1) + 1] = hy[lane]; rh[3 * (lane - 1) + 2] = hz[lane];
    vh[3 * (lane - 1) + 0] = ux[lane]; vh[3 * (lane - 1) + 1] = uy[lane]; vh[3 * (lane - 1) + 2] = uz[lane];
  }
}

template <int NP>
static hipError_t j2h_np(const EphConst& E, const double* rj, const double* vj, double* rh,
                         double* vh, hipStream_t st) {
  hipLaunchKernelGGL(jacobi_to_helio_kernel<NP>, dim3(1), dim3(64), 0, st, E, rj, vj, rh, vh);
  return hipGetLastError();
}

hipError_t launch_jacobi_to_helio(const EphConst& E, const double* rj, const double* vj,
                                  double* rh, double* vh, hipStream_t st) {
  switch (E.np) {
    case 0: return hipSuccess;
    case 1: return j2h_np<1>(E, rj, vj, rh, vh, st);
    case 2: return j2h_np<2>(E, rj, vj, rh, vh, st);
    case 3: return j2h_np<3>(E, rj, vj, rh, vh, st);
    case 4: return j2h_np<4>(E, rj, vj, rh, vh, st);
    case 5: return j2h_np<5>(E, rj, vj, rh, vh, st);
    case 6: return j2h_np<6>(E, rj, vj, rh, vh, st);
    case 7: return j2h_np<7>(E, rj, vj, rh, vh, st);
    case 8: return j2h_np<8>(E, rj, vj, rh, vh, st);
    default: return hipErrorInvalidValue;
  }
}


// Heliocentric -> Jacobi positions or velocities of the planets (one wave):
//   r'_b = r_b - (sum_{k=1}^{b-1} mu_k r_k) / eta_{b-1}.
template <int NP>
__global__ void __launch_bounds__(64)
helio_to_jacobi_kernel(EphConst E, const double* h, double* j) {
  const int lane = threadIdx.x;
  if (lane < 1 || lane > NP) return;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int k = 1; k < lane; ++k) {
    sx = fma_(E.mu[k], h[3 * (k - 1) + 0], sx);
    sy = fma_(E.mu[k], h[3 * (k - 1) + 1], sy);
    sz = fma_(E.mu[k], h[3 * (k - 1) + 2], sz);
  }
  const double ie = E.inv_eta[lane - 1];
  j[3 * (lane - 1) + 0] = fma_(-sx, ie, h[3 * (lane - 1) + 0]);
  j[3 * (lane - 1) + 1] = fma_(-sy, ie, h[3 * (lane - 1) + 1]);
  j[3 * (lane - 1) + 2] = fma_(-sz, ie, h[3 * (lane - 1) + 2]);
}

hipError_t launch_helio_to_jacobi(const EphConst& E, const double* h, double* j, hipStream_t st) {
  switch (E.np) {
    case 0: return hipSuccess;
#define TPM_H2J(N) case N: hipLaunchKernelGGL(helio_to_jacobi_kernel<N>, dim3(1), dim3(64), 0, st, E, h, j); break;
    TPM_H2J(1) TPM_H2J(2) TPM_H2J(3) TPM_H2J(4) TPM_H2J(5) TPM_H2J(6) TPM_H2J(7) TPM_H2J(8)
#undef TPM_H2J
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Sum over particles of the steps spent active in [step_begin, step_end).
__global__ void __launch_bounds__(256)
active_steps_kernel(const int64_t* __restrict__ dstep, int n, int64_t step_begin, int64_t step_end,
                    unsigned long long* acc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  long long v = 0;
  if (i < n) {
    int64_t d = dstep[i];
    int64_t lo = step_begin < step_end ? step_begin : step_end;
    int64_t hi = step_begin < step_end ? step_end : step_begin;
    int64_t e = (d < 0) ? hi : (d < lo ? lo : (d > hi ? hi : d));
    v = e - lo;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, (unsigned long long)v);
}

hipError_t launch_active_steps(const int64_t* dstep, int n, int64_t step_begin, int64_t step_end,
                               unsigned long long* acc, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(active_steps_kernel, dim3((n + 255) / 256), dim3(256), 0, st, dstep, n,
                     step_begin, step_end, acc);
  return hipGetLastError();
}

// ---------------------------------------------------------------- compaction
constexpr int CB = 256;            // threads per compaction block
constexpr int CE = 4;              // elements per thread
constexpr int CTILE = CB * CE;     // elements per block

int compact_scratch_ints(int n_upper) {
  int nb = (n_upper + CTILE - 1) / CTILE;
  return 2 * nb + 2;
}

// Lane prefix count of a 64-bit ballot: number of set bits below this lane.
TPM_DEV int lane_prefix(uint64_t m) {
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
  return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0));
}

__global__ void __launch_bounds__(CB)
compact_count(const int32_t* __restrict__ status, const int32_t* __restrict__ d_nactive,
              int32_t* __restrict__ block_count) {
  const int n = *d_nactive;
  const int base = blockIdx.x * CTILE;
  int c = 0;
#pragma unroll
  for (int e = 0; e < CE; ++e) {
    int i = base + e * CB + threadIdx.x;
    c += (i < n && status[i] == ST_ACTIVE) ? 1 : 0;
  }
  // wave sum by ballots of each bit would be overkill; use a small LDS reduction
  __shared__ int part[CB / 64];
  int wsum = c;
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_down(wsum, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < CB / 64; ++k) t += part[k];
    block_count[blockIdx.x] = t;
  }
}

// Exclusive scan of block counts by one workgroup; writes the new n_active.
__global__ void __launch_bounds__(1024)
compact_scan(const int32_t* __restrict__ block_count, int32_t* __restrict__ block_off, int nb,
             int32_t* __restrict__ d_nactive) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < nb ? block_count[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) block_off[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *d_nactive = carry;
}

__global__ void __launch_bounds__(CB)
compact_scatter(Work src, Work dst, const int32_t* __restrict__ block_off,
                const int32_t* __restrict__ d_nold) {
  const int n_old = *d_nold;
  __shared__ int wcount[CB / 64];
  __shared__ int running;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) running = block_off[blockIdx.x];
  __syncthreads();
  const int base = blockIdx.x * CTILE;
#pragma unroll
  for (int e = 0; e < CE; ++e) {
    int i = base + e * CB + threadIdx.x;
    bool keep = i < n_old && src.status[i] == ST_ACTIVE;
    uint64_t m = __ballot(keep);
    int before = lane_prefix(m);
    if (lane == 0) wcount[wid] = __popcll(m);
    __syncthreads();
    int off = running;
    for (int k = 0; k < wid; ++k) off += wcount[k];
    if (keep) {
      int d = off + before;
      dst.x[d] = src.x[i]; dst.y[d] = src.y[i]; dst.z[d] = src.z[i];
      dst.vx[d] = src.vx[i]; dst.vy[d] = src.vy[i]; dst.vz[d] = src.vz[i];
      dst.slot[d] = src.slot[i];
      dst.status[d] = ST_ACTIVE;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < CB / 64; ++k) t += wcount[k];
      running += t;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) copy_count(const int32_t* a, int32_t* b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *b = *a;
}

hipError_t launch_compact(Work src, Work dst, int32_t* d_nactive, int n_upper, int32_t* scratch,
                          hipStream_t st) {
  int nb = (n_upper + CTILE - 1) / CTILE;
  if (nb <= 0) return hipSuccess;
  int32_t* counts = scratch;
  int32_t* offs = scratch + nb;
  int32_t* n_old = scratch + 2 * nb;
  hipLaunchKernelGGL(copy_count, dim3(1), dim3(64), 0, st, d_nactive, n_old);
  hipLaunchKernelGGL(compact_count, dim3(nb), dim3(CB), 0, st, src.status, d_nactive, counts);
  hipLaunchKernelGGL(compact_scan, dim3(1), dim3(1024), 0, st, counts, offs, nb, d_nactive);
  hipLaunchKernelGGL(compact_scatter, dim3(nb), dim3(CB), 0, st, src, dst, offs, n_old);
  return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
__global__ void __launch_bounds__(256)
finalize_kernel(Work w, const int32_t* __restrict__ d_nactive, Out out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_nactive) return;
  if (w.status[i] != ST_ACTIVE) return;
  const int k = w.slot[i];
  out.r[3 * k + 0] = w.x[i]; out.r[3 * k + 1] = w.y[i]; out.r[3 * k + 2] = w.z[i];
  out.v[3 * k + 0] = w.vx[i]; out.v[3 * k + 1] = w.vy[i]; out.v[3 * k + 2] = w.vz[i];
  out.step[k] = -1;
  out.reason[k] = ST_ACTIVE;
  out.planet[k] = -1;
}

hipError_t launch_finalize(Work w, const int32_t* d_nactive, int n_upper, Out out, hipStream_t st) {
  int grid = (n_upper + 255) / 256;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(256), 0, st, w, d_nactive, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- unit checks
__global__ void sincos_test_kernel(const double* x, double* s, double* c, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ss, cc;
  sincos(x[i], ss, cc);
  s[i] = ss;
  c[i] = cc;
}

hipError_t launch_sincos_test(const double* x, double* s, double* c, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sincos_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, s, c, n);
  return hipGetLastError();
}

__global__ void drift_test_kernel(KepConst K, int kiters, double ftol, const double* in,
                                  double* out, int32_t* ok, int n, double dt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = in[6 * i + 0], y = in[6 * i + 1], z = in[6 * i + 2];
  double vx = in[6 * i + 3], vy = in[6 * i + 4], vz = in[6 * i + 5];
  bool g = drift_fixed(K, dt, kiters, ftol, x, y, z, vx, vy, vz);
  out[6 * i + 0] = x; out[6 * i + 1] = y; out[6 * i + 2] = z;
  out[6 * i + 3] = vx; out[6 * i + 4] = vy; out[6 * i + 5] = vz;
  ok[i] = g ? 1 : 0;
}

hipError_t launch_drift_test(const SysConst& S, const double* rv_in, double* rv_out, int32_t* ok,
                             int n, double dt, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  KepConst K{S.mu0, S.inv_mu0, S.sqrt_mu0, S.inv_sqrt_mu0};
  hipLaunchKernelGGL(drift_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, K, S.kiters,
                     S.ftol, rv_in, rv_out, ok, n, dt);
  return hipGetLastError();
}

}  // namespace tpm
