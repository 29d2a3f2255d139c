// Internal interface between the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpm {

// Wavefronts per SIMD for a particle launch when the caller leaves it to the
// library: as many as the working set's tiles fill on every SIMD alike (at
// least one, at most four).  An uneven split, some SIMDs holding one more
// wavefront than others, lets the tiles on the shared SIMDs fall behind.
inline int auto_waves_per_simd(int ntiles, int ncu) {
  const int per = ntiles / (4 * (ncu > 0 ? ncu : 1));
  return per < 1 ? 1 : (per > 4 ? 4 : per);
}


constexpr int MAX_NP = 8;

// Records msg as this thread's last error (tpm_last_error) and returns code.
int set_error(int code, const char* msg);

// Working set of active particles, structure of arrays (coalesced per lane).
struct Work {
  double* x;
  double* y;
  double* z;
  double* vx;
  double* vy;
  double* vz;
  int32_t* slot;    // index of the particle in the caller's arrays
  int32_t* status;  // 0 while active, else the removal reason
};

// Per-particle results, indexed by slot (caller order).
struct Out {
  double* r;        // [n][3]
  double* v;        // [n][3]
  int64_t* step;    // removal step, -1 while active
  int32_t* reason;
  int32_t* planet;
};

struct KepConst {
  double mu, inv_mu, sqrt_mu, inv_sqrt_mu;
};

struct SysConst {
  int np;
  double mu0, inv_mu0, sqrt_mu0, inv_sqrt_mu0;
  double mu[MAX_NP];
  double rcrit2[MAX_NP];
  double rmax2;          // +inf when escape is off
  int kiters;
  double ftol;
  int universal;         // 1: refused drifts are retried in universal variables
  int handoff;           // 1: within rcrit a particle is handed off, not removed
};

// Particles handed off to the encounter integrator (close-encounter hand-off):
// structure of arrays of capacity n, filled in hand-off order; `step` is the
// global step of each entry's state, `status` ST_ACTIVE or its removal reason.
struct EncList {
  double* x;
  double* y;
  double* z;
  double* vx;
  double* vy;
  double* vz;
  int32_t* slot;
  int32_t* status;
  int64_t* step;
  int32_t* m;            // substeps done in the current step; -1: not yet entered
  int32_t* Ml;           // substeps of the current step
  int32_t* count;        // entries in use
};

// The planet rows of an integrate call for the encounter integrator: chunk c
// covers steps [cb(c), cb(c + 1)) from the call's start, cb(0) = 0,
// cb(1) = k0, cb(c) = k0 + (c - 1) k, cut at nsteps; its rows and its planets'
// velocities are slot c.
struct EncRing {
  const double* rows;    // [slots][ring_rows][3 np + 3]
  const double* vrows;   // [slots][vring_rows][np][3]
  int64_t ring_rows, vring_rows;
  int k0, k;
  int64_t nsteps;
  int64_t step0;         // global step of the call's start
};

// Ephemeris constants (bodies 0..np, body 0 = central mass).
struct EphConst {
  int np;
  double mu[MAX_NP + 1];
  double eta[MAX_NP + 1];       // eta_b = sum_{k<=b} mu_k
  double inv_eta[MAX_NP + 1];   // 1/eta_b
  double mup[MAX_NP + 1];       // Jacobi Kepler constant mu0 eta_b / eta_{b-1}
  double cj[MAX_NP + 1];        // mu_b / eta_b: weight of r'_b in the heliocentric positions
  // squared mutual Hill radius ((mu_i+mu_j)/(3 mu0))^(1/3) (a_i + a_j)/2 with
  // the planets' osculating semi-major axes when they were set
  double hill2[MAX_NP + 1][MAX_NP + 1];
};

// Work-queue bookkeeping of one particle launch (see particle_queue).
struct QueueLaunch {
  unsigned long long* ctr;     // device item counter
  unsigned long long base;     // its value when this launch starts
  uint32_t* progress;          // device per-tile progress counters
  uint32_t epoch;              // their value when this launch starts
  int nsub;                    // sub-chunks per chunk
  int workers;                 // wavefronts launched
  int block;                   // threads per workgroup (multiple of 64)
  int32_t* error;              // device flag set on an over-long wait
  bool deep = false;           // planet rows fetched three steps ahead, not one (for
                               // launches of one wavefront per SIMD)
};

// Particle chunk: nsteps steps through rows[0..nsteps] (row 0 = step0) over
// the first grid_n (>= active count) working-set entries.
hipError_t launch_particle_chunk(const SysConst& S, Work w, const int32_t* d_nactive, int grid_n,
                                 Out out, const double* rows, int nsteps, double dt, int64_t step0,
                                 const QueueLaunch& QL, hipStream_t st);

// Ephemeris chunk: advances the Jacobi state (rj, vj: [np][3]) by nsteps and
// writes rows[0..nsteps]; flag receives the first step of a planet close
// approach (or -2 for an unbound planet) if it is still -1.  vside (may be
// null) receives the heliocentric planet velocities at rows 0 and nsteps,
// [2][np][3].
// vrows (may be null) receives the heliocentric planet velocities of every
// row, [nsteps+1][np][3] (for the encounter integrator's interpolation).
hipError_t launch_ephemeris_chunk(const EphConst& E, double* rj, double* vj, double* rows,
                                  int nsteps, double dt, int64_t step0, int64_t* flag,
                                  hipStream_t st, double* vside = nullptr,
                                  double* vrows = nullptr);

// ---- close-encounter hand-off
// Move the working set's handed-off entries (status >= HANDOFF_BASE, set by
// the particle kernel of the chunk that starts at step0) to the end of the
// encounter list, marking them handed in the working set; snap receives the
// list's new length.
hipError_t launch_handoff_gather(Work w, const int32_t* d_nactive, int n_upper, EncList L,
                                 int64_t step0, int32_t* snap, hipStream_t st);
// Advance the first *snap list entries towards step `target` of the call
// with the encounter reading (plain map steps outside the hand-off radius
// S.rcrit2, M substeps with interpolated planets inside it, removal within
// rrem2, beyond S.rmax2, on a refused drift), at most `budget` micro-steps
// per entry (0: no limit); removals go to `out`.
hipError_t launch_encounter_run(const SysConst& S, const double* rrem2, EncList L,
                                const int32_t* snap, int n_upper, const EncRing& R,
                                int64_t target, int64_t budget, double dt, int M, Out out,
                                hipStream_t st);
// Append the list's active entries to the working set (after its active
// entries, *d_nactive grows) and empty the list.
hipError_t launch_handoff_merge(EncList L, int n_upper, Work w, int32_t* d_nactive,
                                hipStream_t st);

// Stable partition of the working set: active entries of src (in order) go to
// dst; d_nactive is updated in place.  scratch holds >= 2 * nblocks + 1 ints.
hipError_t launch_compact(Work src, Work dst, int32_t* d_nactive, int n_upper, int32_t* scratch,
                          hipStream_t st);
int compact_scratch_ints(int n_upper);

// Write the still-active particles of the working set into out (by slot).
hipError_t launch_finalize(Work w, const int32_t* d_nactive, int n_upper, Out out, hipStream_t st);

// Helio -> Jacobi on the host-side arrays is done in the runtime; conversion of
// the device Jacobi state back to heliocentric r, v:
hipError_t launch_jacobi_to_helio(const EphConst& E, const double* rj, const double* vj,
                                  double* rh, double* vh, hipStream_t st);

hipError_t launch_helio_to_jacobi(const EphConst& E, const double* h, double* j, hipStream_t st);

// Steps spent active in [step_begin, step_end) summed over particles (for a
// backward run the range is taken in absolute order).
hipError_t launch_active_steps(const int64_t* dstep, int n, int64_t step_begin, int64_t step_end,
                               unsigned long long* acc, hipStream_t st);

// ---- many systems in one launch
// Per-system constants of the batched particle kernel (device array).
struct SysDev {
  int np, kiters;
  double ftol, rmax2, dt;
  KepConst K;
  double mu[MAX_NP];
  double rcrit2[MAX_NP];
  int64_t ring_off;      // offset (doubles) of this system's planet-table ring
};

// 64 consecutive working-set entries of one system.
struct TileDesc {
  int32_t sys, first, count, pad;
};

struct BatchQueueArgs {
  unsigned long long* ctr;
  unsigned long long base;
  uint32_t* progress;
  uint32_t epoch;
  int ntiles, nsub, sub_steps, nsteps;
  int64_t step0;
  int slot;
  int64_t slot_rows;     // rows per ring slot (chunk + 1)
  int32_t* error;
  const int32_t* ntiles_dev;   // non-null: the tile count is read here (runs that compact)
};

hipError_t launch_ephemeris_batch(const EphConst* E, double* rj, double* vj, double* ring,
                                  const int64_t* ring_off, int slot, int64_t slot_stride_rows,
                                  int nsys, int nsteps, const double* dt, int64_t step0,
                                  int64_t* flag, hipStream_t st);
hipError_t launch_helio_to_jacobi_batch(const EphConst* E, const double* h, double* j, int nsys,
                                        hipStream_t st);
hipError_t launch_particle_batch(const SysDev* sys, const TileDesc* tiles, Work w, Out out,
                                 const double* ring, const BatchQueueArgs& Q, int workers,
                                 int block, hipStream_t st);
// Rebuild the tiles after a compaction of a batched working set (grouped by
// system): psys[slot] is a particle's system, sorder the systems in queue
// order; start/end are [nsys] scratch; the tile count goes to ntiles_dev.
hipError_t launch_batch_retile(Work w, const int32_t* d_nactive, int n_upper, const int32_t* psys,
                               const int32_t* sorder, int nsys, int32_t* start, int32_t* end,
                               TileDesc* tiles, int32_t* ntiles_dev, hipStream_t st);
// Zero a work-queue item counter (a kernel, so it can sit in a captured graph).
hipError_t launch_queue_reset(unsigned long long* ctr, hipStream_t st);

// Unit checks of the device math (test entry points).
hipError_t launch_sincos_test(const double* x, double* s, double* c, int n, hipStream_t st);
hipError_t launch_rsqrt_test(const double* x, double* out, int n, hipStream_t st);
// S.universal: 0 fixed-iteration drift, 1 with the universal fallback, 2
// universal drift alone.
hipError_t launch_drift_test(const SysConst& S, const double* rv_in, double* rv_out, int32_t* ok,
                             int n, double dt, hipStream_t st);

}  // namespace tpm
