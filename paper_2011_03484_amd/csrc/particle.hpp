// Per-particle pieces of the test-particle map (Zhang & Gladman 2021, sec. 2.2).
#pragma once
#include "kepler.hpp"

namespace tpm {

enum : int32_t { ST_ACTIVE = 0, ST_ENCOUNTER = 1, ST_ESCAPE = 2, ST_KEPLER = 3 };
// Working-set states of the close-encounter hand-off (never in results):
// HANDOFF_BASE + t, handed off at local step t of the current chunk; ST_HANDED,
// moved to the encounter list.
constexpr int32_t ST_HANDED = 4;
constexpr int32_t HANDOFF_BASE = 16;

// Planet constants of one system, passed by value so they land in SGPRs.
template <int NP>
struct PlanetConst {
  double mu[NP > 0 ? NP : 1];
  double rcrit2[NP > 0 ? NP : 1];
};

// One planet-table row (r_1..r_NP, h0) held in VGPRs.
template <int NP>
struct Row {
  double v[3 * NP + 3];
};

// A zero the compiler cannot see through, in a VGPR.  Added to a wave-uniform
// address it turns the row's loads into vector loads (one broadcast request
// per load): the row then lands in VGPRs, which can hold the next row while
// the current step runs, instead of in SGPRs, which are fully used.
TPM_DEV int opaque_zero_vgpr() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// Load a row into VGPRs (issued early; the first use waits for it).
template <int NP>
TPM_DEV void load_row(Row<NP>& R, const double* __restrict__ row, int zero) {
#pragma unroll
  for (int k = 0; k < 3 * NP + 3; ++k) R.v[k] = row[zero + k];
}

// A kernel's argument segment, read where a value is used: a kernel that
// reads rarely used pointer arguments (records, an item's start and end)
// through karg_field keeps them out of the scalar registers its loops need.
// The address is hidden from the compiler at each use, so the load stays
// there instead of being hoisted to the kernel's start.  The offsets come
// from a struct with the kernel's leading parameters in order, which the
// argument segment lays out as a C struct.  (The host pass of these sources
// compiles no device code from them.)
typedef const __attribute__((address_space(4))) char* KargPtr;

TPM_DEV KargPtr karg_at_use(KargPtr p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <typename T>
TPM_DEV T karg_field(KargPtr p, size_t off) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *reinterpret_cast<const __attribute__((address_space(4))) T*>(karg_at_use(p) + off);
#else
  (void)p;
  (void)off;
  return T{};
#endif
}

// Kick acceleration from one table row (sec. 2.2, kick equation):
//   a = h0 - sum_j mu_j d_j / |d_j|^3,   d_j = r - r_j,
// and the encounter test |d_j| < rcrit_j (lowest j wins; -1 if none).
// The row (3 NP + 3 doubles: r_1..r_NP, h0) is the same for every lane.
template <int NP, typename RowT>
TPM_DEV int accel(const RowT& row, const PlanetConst<NP>& P,
                  double x, double y, double z, double& ax, double& ay, double& az) {
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
    // to rounding (the first-order form, good to 2^-45, is always a little
    // low: a bias of the same sign in every kick)
    double k = mul_rsqrt3(P.mu[j], d2);
    ax = fma_(-k, dx, ax);
    ay = fma_(-k, dy, ay);
    az = fma_(-k, dz, az);
  }
  // lowest planet index inside its radius: scanning downwards, the last hit
  // wins (one compare per planet, no combined lane predicates)
  int hit = -1;
#pragma unroll
  for (int j = NP - 1; j >= 0; --j) hit = d2s[j] < P.rcrit2[j] ? j : hit;
  return hit;
}

}  // namespace tpm
