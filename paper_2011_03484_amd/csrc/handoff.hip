// Close-encounter hand-off (Zhang & Gladman 2021, sec. 5: particles in close
// encounters move off the main integration, so the bulk keeps its uniform,
// full-speed kernel).  The method of the encounter integration is this
// library's reading, applied identically by the oracle:
//
//  * at every step boundary a particle within the hand-off radius rcrit_j of
//    any planet takes its next step as an encounter step, any other particle
//    the plain map step;
//  * an encounter step is M equal substeps h = dt/M of the same kick - drift -
//    kick, with the planets between the two table rows on the cubic Hermite
//    interpolant of their heliocentric positions and velocities (the row
//    values themselves at the step's two ends) and h0 = -sum_j mu_j r_j/|r_j|^3
//    of the interpolated positions;
//  * removal within the removal radius rrem_j at any step or substep boundary
//    (lowest j; step n at a step boundary, n + 1 at a substep inside step n,
//    keeping that substep's state), beyond rmax at a step boundary, or on a
//    refused drift (the state at the start of the failing substep, step n).
//
// The particle kernel hands a lane off where it would otherwise record an
// encounter removal (hand-off radius = its rcrit) and leaves its state in the
// working set; handoff_gather moves such entries to the encounter list;
// encounter_run advances the list towards the end of a chunk, one lane per
// entry (the lanes diverge, which is why they left the main kernel);
// handoff_merge puts the survivors back into the working set at the end of
// an integrate call.  A lane may lag behind the main kernel: every launch
// gives it a budget of micro-steps, and where it stops (at a step or substep
// boundary) the next launch resumes it, with the planet rows of every chunk
// of the call still in place; the last launch of a call has no budget.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "particle.hpp"
#include "universal.hpp"

namespace tpm {

__global__ void __launch_bounds__(256)
handoff_gather(Work w, const int32_t* __restrict__ d_nactive, EncList L, int64_t step0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_nactive) return;
  const int32_t st = w.status[i];
  if (st < HANDOFF_BASE) return;
  const int k = atomicAdd(L.count, 1);
  L.x[k] = w.x[i]; L.y[k] = w.y[i]; L.z[k] = w.z[i];
  L.vx[k] = w.vx[i]; L.vy[k] = w.vy[i]; L.vz[k] = w.vz[i];
  L.slot[k] = w.slot[i];
  L.status[k] = ST_ACTIVE;
  L.step[k] = step0 + (st - HANDOFF_BASE);
  L.m[k] = -1;                            // not yet checked at its hand-off boundary
  w.status[i] = ST_HANDED;
}

__global__ void __launch_bounds__(64) handoff_snap(const int32_t* count, int32_t* snap) {
  if (threadIdx.x == 0) *snap = *count;
}

hipError_t launch_handoff_gather(Work w, const int32_t* d_nactive, int n_upper, EncList L,
                                 int64_t step0, int32_t* snap, hipStream_t st) {
  if (n_upper > 0)
    hipLaunchKernelGGL(handoff_gather, dim3((n_upper + 255) / 256), dim3(256), 0, st, w, d_nactive,
                       L, step0);
  hipLaunchKernelGGL(handoff_snap, dim3(1), dim3(64), 0, st, L.count, snap);
  return hipGetLastError();
}

template <int NP>
struct EncArgs {
  PlanetConst<NP> Prem;   // mu and the removal radii squared
  double renc2[NP > 0 ? NP : 1];
  KepConst K;
  double rmax2, ftol, dt;
  int kiters, M, universal;
  int64_t target;         // step (from the call's start) the lanes advance to
  int64_t budget;         // micro-steps per lane in this launch; 0 = no limit
};

// The kick acceleration from a table row with the particle kernel's
// arithmetic (accel in particle.hpp), returning the lowest planet index within
// its removal radius (or -1) and setting enc when the particle lies within a
// hand-off radius: the two tests share the squared distances.
template <int NP, typename RowT>
TPM_DEV int accel_enc(const RowT& row, const EncArgs<NP>& A, double x, double y, double z,
                      double& ax, double& ay, double& az, bool& enc) {
  ax = row[3 * NP + 0];
  ay = row[3 * NP + 1];
  az = row[3 * NP + 2];
  double d2s[NP > 0 ? NP : 1];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double dx = x - row[3 * j + 0];
    double dy = y - row[3 * j + 1];
    double dz = z - row[3 * j + 2];
    double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
    d2s[j] = d2;
    double k = mul_rsqrt3(A.Prem.mu[j], d2);
    ax = fma_(-k, dx, ax);
    ay = fma_(-k, dy, ay);
    az = fma_(-k, dz, az);
  }
  int hit = -1;
  enc = false;
#pragma unroll
  for (int j = NP - 1; j >= 0; --j) {
    hit = d2s[j] < A.Prem.rcrit2[j] ? j : hit;
    enc = enc | (d2s[j] < A.renc2[j]);
  }
  return hit;
}

// Acceleration at fraction tau of the step from row a to row b (planet
// velocities va, vb per row) with the planets on their Hermite interpolants;
// returns the lowest planet index within its removal radius, or -1.
template <int NP, typename RowA, typename RowB>
TPM_DEV int interp_accel(const EncArgs<NP>& A, double tau, const RowA& ra,
                         const double* __restrict__ va, const RowB& rb,
                         const double* __restrict__ vb, double x, double y, double z, double& ax,
                         double& ay, double& az) {
  const double t2 = tau * tau, t3 = t2 * tau;
  const double h00 = fma_(2.0, t3, fma_(-3.0, t2, 1.0));
  const double h10 = fma_(-2.0, t2, t3 + tau);
  const double h01 = fma_(-2.0, t3, 3.0 * t2);
  const double h11 = t3 - t2;
  const double d10 = h10 * A.dt, d11 = h11 * A.dt;
  double p[NP > 0 ? NP : 1][3];
  ax = 0.0; ay = 0.0; az = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      p[j][c] = fma_(h00, ra[3 * j + c],
                     fma_(d10, va[3 * j + c], fma_(h01, rb[3 * j + c], d11 * vb[3 * j + c])));
    // h0: -mu_j r_j / |r_j|^3
    const double k0 = mul_rsqrt3(A.Prem.mu[j],
                                 fma_(p[j][0], p[j][0], fma_(p[j][1], p[j][1], p[j][2] * p[j][2])));
    ax = fma_(-k0, p[j][0], ax);
    ay = fma_(-k0, p[j][1], ay);
    az = fma_(-k0, p[j][2], az);
  }
  int hit = -1;
#pragma unroll
  for (int j = NP - 1; j >= 0; --j) {
    const double dx = x - p[j][0], dy = y - p[j][1], dz = z - p[j][2];
    const double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
    hit = d2 < A.Prem.rcrit2[j] ? j : hit;
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const double dx = x - p[j][0], dy = y - p[j][1], dz = z - p[j][2];
    const double k = mul_rsqrt3(A.Prem.mu[j], fma_(dx, dx, fma_(dy, dy, dz * dz)));
    ax = fma_(-k, dx, ax);
    ay = fma_(-k, dy, ay);
    az = fma_(-k, dz, az);
  }
  return hit;
}

// The drift of a step or substep: the fixed-count elliptic solve, retried in
// universal variables where it is refused and the option is on (the same
// arithmetic as the particle kernel's step).
template <int NP, int KIT>
TPM_DEV bool enc_drift(const EncArgs<NP>& A, double dt, double& x, double& y, double& z,
                       double& vx, double& vy, double& vz) {
  double nx = x, ny = y, nz = z, nvx = vx, nvy = vy, nvz = vz;
  bool ok = drift_fixed(A.K, dt, KIT > 0 ? KIT : A.kiters, A.ftol, nx, ny, nz, nvx, nvy, nvz);
  if (!ok && A.universal) {
    nx = x; ny = y; nz = z; nvx = vx; nvy = vy; nvz = vz;
    ok = drift_universal(A.K.mu, dt, nx, ny, nz, nvx, nvy, nvz);
  }
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return ok;
}

// One lane per list entry.  Each lane runs its own sequence of micro-steps,
// a plain step (one kick - drift - kick of dt) or one substep of an encounter
// step (of dt / M), so a lane in an encounter costs its wavefront M
// micro-steps per step and the others go on with their plain steps meanwhile:
// a wavefront takes max over its lanes of (plain steps + M x encounter steps)
// iterations, not M per step whenever any lane is in an encounter.  The
// acceleration at the end of a plain step or of a step's last substep comes
// from the row itself (exactly the main kernel's arithmetic), inside a step
// from the interpolated planets.  The closing row of a lane's step stays in
// registers through its substeps, each micro-step fetches the next one's, and
// the hand-off radius test of a step boundary comes with the acceleration
// there.  A lane enters at a step boundary (its hand-off boundary, a chunk's
// first step, or where a budget stopped it) as the particle kernel enters a
// chunk: acceleration, removal-radius and escape checks from the row there;
// inside a step (a budget stopped it after a substep) with the acceleration of
// the interpolated planets there.  Either gives the values the lane had when
// it stopped, bit for bit.  KIT > 0 fixes the Newton count at compile time,
// as in the particle kernel.
// encounter_run's parameters in order, for the offsets of the list and the
// results in its argument segment (see karg_field).
template <int NP>
struct EncRunArgs {
  EncArgs<NP> A;
  EncList L;
  const int32_t* snap;
  EncRing R;
  Out out;
};

template <int NP, int KIT>
__global__ void __launch_bounds__(64)
encounter_run(EncArgs<NP> A, EncList L_arg, const int32_t* __restrict__ snap, EncRing R,
              Out out_arg) {
  constexpr int ROW = 3 * NP + 3;
  // the list's and the results' pointers are read where they are used (the
  // entry, a removal, the exit), which leaves the micro-step loop's scalar
  // registers to its constants
  (void)L_arg;
  (void)out_arg;
  const KargPtr ka = (KargPtr)__builtin_amdgcn_kernarg_segment_ptr();
  auto list = [&]() { return karg_field<EncList>(ka, offsetof(EncRunArgs<NP>, L)); };
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *snap) return;
  const EncList L = list();
  if (L.status[i] != ST_ACTIVE) return;
  // chunk c covers steps [cb(c), cb(c + 1)) of the call, cut at its end
  auto cb = [&](int c) -> int64_t {
    const int64_t b = c == 0 ? 0 : R.k0 + (int64_t)(c - 1) * R.k;
    return b < R.nsteps ? b : R.nsteps;
  };
  const int64_t g0 = L.step[i] - R.step0;
  if (g0 < 0 || g0 > R.nsteps) return;   // not in this call (never the case)
  int m = L.m[i], Ml = L.Ml[i];
  if (m > 0 && g0 >= R.nsteps) return;   // inside a step past the call's end (never the case)
  auto chunk_of = [&](int64_t g) -> int { return g < R.k0 ? 0 : 1 + (int)((g - R.k0) / R.k); };
  // a lane inside step g0 (a budget stopped it after a substep) is in the
  // chunk that holds that step; a lane at the boundary g0 in the chunk that
  // ends at or holds it: at a chunk's end it enters with that chunk's last
  // row (the next chunk's rows may not exist yet when g0 is the launch's
  // start)
  int c = m > 0 ? chunk_of(g0) : (g0 == 0 ? 0 : chunk_of(g0 - 1));
  int s = (int)(g0 - cb(c));
  int ks = (int)(cb(c + 1) - cb(c));
  const double* rc = R.rows + (size_t)c * R.ring_rows * ROW;
  const double* vc = R.vrows + (size_t)c * R.vring_rows * 3 * NP;
  double x = L.x[i], y = L.y[i], z = L.z[i];
  double vx = L.vx[i], vy = L.vy[i], vz = L.vz[i];
  auto remove = [&](int32_t why, int64_t st, int32_t pl, double rx, double ry, double rz,
                    double ux, double uy, double uz) {
    const EncList Lr = list();
    const Out out = karg_field<Out>(ka, offsetof(EncRunArgs<NP>, out));
    const int k = Lr.slot[i];
    out.r[3 * k + 0] = rx; out.r[3 * k + 1] = ry; out.r[3 * k + 2] = rz;
    out.v[3 * k + 0] = ux; out.v[3 * k + 1] = uy; out.v[3 * k + 2] = uz;
    out.step[k] = st;
    out.reason[k] = why;
    out.planet[k] = pl;
    Lr.status[i] = why;
  };
  double ax, ay, az;
  bool enc = false;         // within a hand-off radius at the current step boundary
  // entry at step boundary s of chunk c: acceleration, removal radius, escape
  auto enter = [&]() -> bool {
    Row<NP> R0;
    load_row<NP>(R0, rc + (size_t)s * ROW, 0);
    const int hit = accel_enc<NP>(R0.v, A, x, y, z, ax, ay, az, enc);
    if (hit >= 0) {
      remove(ST_ENCOUNTER, R.step0 + cb(c) + s, hit, x, y, z, vx, vy, vz);
      return false;
    }
    if (fma_(x, x, fma_(y, y, z * z)) > A.rmax2) {
      remove(ST_ESCAPE, R.step0 + cb(c) + s, -1, x, y, z, vx, vy, vz);
      return false;
    }
    return true;
  };
  if (m <= 0) {
    m = 0;
    if (!enter()) return;
  } else {
    const double* va = vc + (size_t)s * 3 * NP;
    interp_accel<NP>(A, (double)m / Ml, rc + (size_t)s * ROW, va, rc + (size_t)(s + 1) * ROW,
                     va + 3 * NP, x, y, z, ax, ay, az);
  }
  // into the next chunk at chunk c's end, entered as the particle kernel
  // enters a chunk
  auto next_chunk = [&]() -> bool {
    ++c;
    s = 0;
    ks = (int)(cb(c + 1) - cb(c));
    rc = R.rows + (size_t)c * R.ring_rows * ROW;
    vc = R.vrows + (size_t)c * R.vring_rows * 3 * NP;
    return enter();
  };
  const double hM = A.dt / A.M;
  int64_t used = 0;
  if (cb(c) + s < A.target) {
    if (s == ks && !next_chunk()) return;
    Row<NP> Rb, Rn;         // the closing row of this and of the next micro-step
    load_row<NP>(Rb, rc + (size_t)(s + 1) * ROW, 0);
    for (;;) {
      if (A.budget > 0 && used >= A.budget) break;
      // the mode of a step is decided at its first boundary
      if (m == 0) Ml = enc ? A.M : 1;
      // the closing row of the next micro-step, fetched by every lane (row
      // s + 2 if this micro-step ends the step, else row s + 1 again) so
      // that the loads are not conditional and their latency hides behind
      // the drift
      const bool ends = m + 1 == Ml;
      load_row<NP>(Rn, rc + (size_t)min(s + (ends ? 2 : 1), ks) * ROW, 0);
      const double h = Ml == 1 ? A.dt : hM;
      const double hh = 0.5 * h;
      double nx = x, ny = y, nz = z;
      double nvx = fma_(hh, ax, vx), nvy = fma_(hh, ay, vy), nvz = fma_(hh, az, vz);
      if (!enc_drift<NP, KIT>(A, h, nx, ny, nz, nvx, nvy, nvz)) {
        // the state at the start of the failing (sub)step
        remove(ST_KEPLER, R.step0 + cb(c) + s, -1, x, y, z, vx, vy, vz);
        return;
      }
      int hit;
      if (ends) {
        hit = accel_enc<NP>(Rb.v, A, nx, ny, nz, ax, ay, az, enc);
      } else {
        const double* va = vc + (size_t)s * 3 * NP;
        hit = interp_accel<NP>(A, (double)(m + 1) / Ml, rc + (size_t)s * ROW, va, Rb.v,
                               va + 3 * NP, nx, ny, nz, ax, ay, az);
      }
      x = nx; y = ny; z = nz;
      vx = fma_(hh, ax, nvx); vy = fma_(hh, ay, nvy); vz = fma_(hh, az, nvz);
      if (hit >= 0) {
        // step n + 1 at the step's end or at a substep inside it
        remove(ST_ENCOUNTER, R.step0 + cb(c) + s + 1, hit, x, y, z, vx, vy, vz);
        return;
      }
      Rb = Rn;
      ++used;
      if (++m == Ml) {
        m = 0;
        ++s;
        if (fma_(x, x, fma_(y, y, z * z)) > A.rmax2) {
          remove(ST_ESCAPE, R.step0 + cb(c) + s, -1, x, y, z, vx, vy, vz);
          return;
        }
        if (cb(c) + s >= A.target) break;
        if (s == ks) {
          if (!next_chunk()) return;
          load_row<NP>(Rb, rc + ROW, 0);
        }
      }
    }
  }
  const EncList Le = list();
  Le.x[i] = x; Le.y[i] = y; Le.z[i] = z;
  Le.vx[i] = vx; Le.vy[i] = vy; Le.vz[i] = vz;
  Le.step[i] = R.step0 + cb(c) + s;
  Le.m[i] = m;
  Le.Ml[i] = Ml;
}

template <int NP>
static hipError_t enc_np(const SysConst& S, const double* rrem2, EncList L, const int32_t* snap,
                         int n_upper, const EncRing& R, int64_t target, int64_t budget, double dt,
                         int M, Out out, hipStream_t st) {
  EncArgs<NP> A;
  for (int j = 0; j < (NP > 0 ? NP : 1); ++j) {
    A.Prem.mu[j] = NP > 0 ? S.mu[j] : 0.0;
    A.Prem.rcrit2[j] = NP > 0 ? rrem2[j] : 0.0;
    A.renc2[j] = NP > 0 ? S.rcrit2[j] : 0.0;
  }
  A.K = KepConst{S.mu0, S.inv_mu0, S.sqrt_mu0, S.inv_sqrt_mu0};
  A.rmax2 = S.rmax2;
  A.ftol = S.ftol;
  A.dt = dt;
  A.kiters = S.kiters;
  A.M = M;
  A.universal = S.universal;
  A.target = target;
  A.budget = budget;
  if (S.kiters == 5)
    hipLaunchKernelGGL((encounter_run<NP, 5>), dim3((n_upper + 63) / 64), dim3(64), 0, st, A, L,
                       snap, R, out);
  else
    hipLaunchKernelGGL((encounter_run<NP, 0>), dim3((n_upper + 63) / 64), dim3(64), 0, st, A, L,
                       snap, R, out);
  return hipGetLastError();
}

hipError_t launch_encounter_run(const SysConst& S, const double* rrem2, EncList L,
                                const int32_t* snap, int n_upper, const EncRing& R,
                                int64_t target, int64_t budget, double dt, int M, Out out,
                                hipStream_t st) {
  if (n_upper <= 0) return hipSuccess;
  if (M < 1 || R.k0 < 1 || R.k < 1 || target < 0 || target > R.nsteps)
    return hipErrorInvalidValue;
  switch (S.np) {
#define TPM_ENC(N) \
    case N: return enc_np<N>(S, rrem2, L, snap, n_upper, R, target, budget, dt, M, out, st);
    TPM_ENC(0) TPM_ENC(1) TPM_ENC(2) TPM_ENC(3) TPM_ENC(4) TPM_ENC(5) TPM_ENC(6) TPM_ENC(7)
    TPM_ENC(8)
#undef TPM_ENC
    default: return hipErrorInvalidValue;
  }
}

__global__ void __launch_bounds__(256)
handoff_merge(EncList L, int n_upper, Work w, int32_t* __restrict__ d_nactive) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_upper || i >= *L.count || L.status[i] != ST_ACTIVE) return;
  const int k = atomicAdd(d_nactive, 1);
  w.x[k] = L.x[i]; w.y[k] = L.y[i]; w.z[k] = L.z[i];
  w.vx[k] = L.vx[i]; w.vy[k] = L.vy[i]; w.vz[k] = L.vz[i];
  w.slot[k] = L.slot[i];
  w.status[k] = ST_ACTIVE;
}

__global__ void __launch_bounds__(64) handoff_clear(int32_t* count) {
  if (threadIdx.x == 0) *count = 0;
}

hipError_t launch_handoff_merge(EncList L, int n_upper, Work w, int32_t* d_nactive,
                                hipStream_t st) {
  if (n_upper > 0)
    hipLaunchKernelGGL(handoff_merge, dim3((n_upper + 255) / 256), dim3(256), 0, st, L, n_upper, w,
                       d_nactive);
  hipLaunchKernelGGL(handoff_clear, dim3(1), dim3(64), 0, st, L.count);
  return hipGetLastError();
}

}  // namespace tpm
