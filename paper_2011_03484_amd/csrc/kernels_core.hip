// Core kernels of the test-particle map on gfx950 (FP64 throughout).
//
//  * particle_queue  - one lane per particle; the particle stays in registers
//    for hundreds of steps (sec. 2.2: a single kernel loops over the planet
//    chunk so each particle is read and written once per chunk), with the
//    chunk's (tile, sub-chunk) items handed out dynamically to wavefronts.
//    Every lane reads the same planet-table row: broadcast vector loads into
//    VGPRs, one step ahead of its use.
//  * ephemeris_chunk - one wavefront; lane b holds Jacobi body b.  Wisdom-Holman
//    kick-drift-kick of the planets (sec. 2.2, planet integration) writing the
//    heliocentric positions and the indirect term h0 per step.
//  * compact_*       - stable partition of the working set so removed particles
//    stop occupying lanes (sec. 2.2, resync interval), by wave ballots, an LDS
//    scan and ordered block offsets.
//  * finalize        - scatter the active particles back to caller order.
#include "internal.h"
#include "particle.hpp"
#include "universal.hpp"

namespace tpm {

// ---------------------------------------------------------------- particles
template <int NP>
struct ChunkArgs {
  PlanetConst<NP> P;
  KepConst K;
  double rmax2, ftol, dt;
  int kiters, nsteps;
  int64_t step0;
  int handoff;   // within rcrit: hand off to the encounter integrator, not removal
};

// The work-queue kernel's leading arguments as its argument segment lays them
// out (particle_queue: w, d_nactive, out, ...); see karg_field.
struct QueueArgsHead {
  Work w;
  const int32_t* n;
  Out out;
};
TPM_DEV Work karg_work(KargPtr p) { return karg_field<Work>(p, offsetof(QueueArgsHead, w)); }
TPM_DEV Out karg_out(KargPtr p) { return karg_field<Out>(p, offsetof(QueueArgsHead, out)); }

// Advance particle i of the working set through steps [s_begin, s_end) of a
// chunk whose rows start at `rows` (row k = step step0 + k; all rows of the
// chunk are written before the launch).  The step loop is uniform across the
// wavefront (s_begin, s_end are wave-uniform); removed lanes are masked off
// and the wavefront leaves early once none is active.  KIT > 0 fixes the
// Newton count at compile time; DEPTH > 0 fetches each planet row DEPTH
// steps ahead into VGPRs (for launches with a few wavefronts per SIMD; 0:
// scalar loads at the point of use, for many).
//
// UNIV: a drift the fixed-iteration solve refuses is taken in universal
// variables instead (drift_universal); the particle is removed as KEPLER only
// if that gives no finite result either.
// KA: w and out are read from the work-queue kernel's argument segment ka
// where they are used (the item's start and end, a record), which leaves the
// step loop's scalar registers to its constants.
template <int NP, int KIT, int DEPTH, bool UNIV = false, bool KA = false>
TPM_DEV void advance(Work w, Out out, const double* __restrict__ rows, const ChunkArgs<NP>& A,
                     int i, bool valid, int s_begin, int s_end, KargPtr ka = nullptr) {
  constexpr int ROW = 3 * NP + 3;
  const int kiters = KIT > 0 ? KIT : A.kiters;
  if (KA) w = karg_work(ka);
  valid = valid && w.status[i] == ST_ACTIVE;
  double x = 0, y = 0, z = 0, vx = 0, vy = 0, vz = 0;
  if (valid) {
    x = w.x[i]; y = w.y[i]; z = w.z[i];
    vx = w.vx[i]; vy = w.vy[i]; vz = w.vz[i];
  }
  // A lane's removal record (the state it keeps, step, reason, planet) is
  // written out in the step that removes it, so the state registers can be
  // overwritten unconditionally; a removed lane takes no further part.  With
  // the hand-off on, a lane within a planet's radius is handed off instead:
  // its state stays in the working set, marked with its local step, for the
  // encounter integrator.
  int32_t reason = valid ? ST_ACTIVE : -1;
  auto record = [&](int32_t why, int64_t st, int32_t pl, double rx, double ry, double rz,
                    double ux, double uy, double uz) {
    const Work wr = KA ? karg_work(ka) : w;
    if (A.handoff && why == ST_ENCOUNTER) {
      wr.x[i] = rx; wr.y[i] = ry; wr.z[i] = rz;
      wr.vx[i] = ux; wr.vy[i] = uy; wr.vz[i] = uz;
      reason = HANDOFF_BASE + (int32_t)(st - A.step0);
      wr.status[i] = reason;
      return;
    }
    const Out o = KA ? karg_out(ka) : out;
    const int k = wr.slot[i];
    o.r[3 * k + 0] = rx; o.r[3 * k + 1] = ry; o.r[3 * k + 2] = rz;
    o.v[3 * k + 0] = ux; o.v[3 * k + 1] = uy; o.v[3 * k + 2] = uz;
    o.step[k] = st;
    o.reason[k] = why;
    o.planet[k] = pl;
    wr.status[i] = why;
    reason = why;
  };
  double ax, ay, az;
  int hit = accel<NP>(rows + (size_t)s_begin * ROW, A.P, x, y, z, ax, ay, az);
  if (valid) {
    if (hit >= 0) record(ST_ENCOUNTER, A.step0 + s_begin, hit, x, y, z, vx, vy, vz);
    else if (fma_(x, x, fma_(y, y, z * z)) > A.rmax2)
      record(ST_ESCAPE, A.step0 + s_begin, -1, x, y, z, vx, vy, vz);
  }
  const double h = 0.5 * A.dt;
  // one step s -> s + 1, with the row that ends it (row s + 1)
  auto step = [&](int s, const auto& row) {
    if (reason == ST_ACTIVE) {
      double nx = x, ny = y, nz = z;
      double nvx = fma_(h, ax, vx), nvy = fma_(h, ay, vy), nvz = fma_(h, az, vz);
      bool ok = drift_fixed(A.K, A.dt, kiters, A.ftol, nx, ny, nz, nvx, nvy, nvz);
      if (UNIV && !wave_all(ok)) {
        if (!ok) {
          nx = x; ny = y; nz = z;
          nvx = fma_(h, ax, vx); nvy = fma_(h, ay, vy); nvz = fma_(h, az, vz);
          ok = drift_universal(A.K.mu, A.dt, nx, ny, nz, nvx, nvy, nvz);
        }
      }
      double bx, by, bz;
      const int hit1 = accel<NP>(row, A.P, nx, ny, nz, bx, by, bz);
      const double r2 = fma_(nx, nx, fma_(ny, ny, nz * nz));
      nvx = fma_(h, bx, nvx); nvy = fma_(h, by, nvy); nvz = fma_(h, bz, nvz);
      if (!ok | (hit1 >= 0) | (r2 > A.rmax2)) {
        // a Kepler failure keeps the state at the start of the step
        if (!ok) record(ST_KEPLER, A.step0 + s, -1, x, y, z, vx, vy, vz);
        else if (hit1 >= 0) record(ST_ENCOUNTER, A.step0 + s + 1, hit1, nx, ny, nz, nvx, nvy, nvz);
        else record(ST_ESCAPE, A.step0 + s + 1, -1, nx, ny, nz, nvx, nvy, nvz);
      }
      x = nx; y = ny; z = nz;
      vx = nvx; vy = nvy; vz = nvz;
      ax = bx; ay = by; az = bz;
    }
  };
  // leave once every lane is removed (checked every 8 steps: the check itself
  // costs a vector-to-scalar round trip)
  auto all_removed = [&](int s) {
    return ((s - s_begin) & 7) == 0 && wave_all(reason != ST_ACTIVE);
  };
  if (DEPTH == 1) {
    // The row that ends step s is fetched during step s - 1, into the one of
    // two alternating VGPR buffers that step s - 1 does not use: with few
    // wavefronts per SIMD nothing else hides that load's latency.
    const int zero = opaque_zero_vgpr();
    Row<NP> ra, rb;
    load_row<NP>(ra, rows + (size_t)(s_begin + 1) * ROW, zero);
    for (int s = s_begin; s < s_end; s += 2) {
      if (all_removed(s)) break;
      load_row<NP>(rb, rows + (size_t)min(s + 2, s_end) * ROW, zero);
      step(s, ra.v);
      if (s + 1 >= s_end) break;
      load_row<NP>(ra, rows + (size_t)min(s + 3, s_end) * ROW, zero);
      step(s + 1, rb.v);
    }
  } else if (DEPTH == 3) {
    // Three steps ahead, four buffers in turn: with one wavefront per SIMD
    // the particles run right behind the planet map, and a row just written
    // on another die can take longer than a step to arrive.
    const int zero = opaque_zero_vgpr();
    Row<NP> ra, rb, rc, rd;
    load_row<NP>(ra, rows + (size_t)(s_begin + 1) * ROW, zero);
    load_row<NP>(rb, rows + (size_t)min(s_begin + 2, s_end) * ROW, zero);
    load_row<NP>(rc, rows + (size_t)min(s_begin + 3, s_end) * ROW, zero);
    for (int s = s_begin; s < s_end; s += 4) {
      if (all_removed(s)) break;
      load_row<NP>(rd, rows + (size_t)min(s + 4, s_end) * ROW, zero);
      step(s, ra.v);
      if (s + 1 >= s_end) break;
      load_row<NP>(ra, rows + (size_t)min(s + 5, s_end) * ROW, zero);
      step(s + 1, rb.v);
      if (s + 2 >= s_end) break;
      load_row<NP>(rb, rows + (size_t)min(s + 6, s_end) * ROW, zero);
      step(s + 2, rc.v);
      if (s + 3 >= s_end) break;
      load_row<NP>(rc, rows + (size_t)min(s + 7, s_end) * ROW, zero);
      step(s + 3, rd.v);
    }
  } else {
    // many wavefronts per SIMD: rows by scalar loads at their use
    for (int s = s_begin; s < s_end; ++s) {
      if (all_removed(s)) break;
      step(s, rows + (size_t)(s + 1) * ROW);
    }
  }
  if (reason == ST_ACTIVE) {
    const Work we = KA ? karg_work(ka) : w;
    we.x[i] = x; we.y[i] = y; we.z[i] = z;
    we.vx[i] = vx; we.vy[i] = vy; we.vz[i] = vz;
  }
}

// Work queue of one chunk: item = (sub-chunk s, tile t) in s-major order,
// tile = 64 consecutive working-set entries (one wavefront).  Wavefronts take
// items from a monotonic counter, so a wavefront that shares its SIMD with
// other work (or sits alone on one) simply takes fewer items.  Item (s, t)
// waits for item (s-1, t) through a per-tile progress counter; that item was
// taken earlier by a running wavefront, so the wait always ends.  A wait
// longer than the spin limit flags an error and drops the item.
struct QueueArgs {
  unsigned long long* ctr;     // monotonic item counter
  unsigned long long base;     // counter value at this launch's start
  uint32_t* progress;          // per tile: sub-chunks completed (monotonic over launches)
  uint32_t epoch;              // progress value of every tile at this launch's start
  int ntiles, nsub, sub_steps, nsteps;
  int32_t* error;
};

constexpr uint32_t SPIN_LIMIT = 1u << 22;   // about 4 s of polling

TPM_DEV unsigned long long wave_uniform(unsigned long long v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// No part of the item loop runs on a subset of the lanes: the grab, the wait
// and the publish are executed by the whole wavefront (lane 0 alone adds 1 to
// the counter), so the readfirstlane that makes their results wave-uniform
// always sees the full wavefront and the loop's branches stay scalar.
template <int NP, int KIT, bool UNIV, int DEPTH>
__global__ void __launch_bounds__(256)
particle_queue(Work w, const int32_t* __restrict__ d_nactive, Out out,
               const double* __restrict__ rows, ChunkArgs<NP> A, QueueArgs Q) {
  const int lane = threadIdx.x & 63;
  const int n = *d_nactive;
  const unsigned long long total = (unsigned long long)Q.ntiles * Q.nsub;
  const unsigned long long one = lane == 0 ? 1ull : 0ull;
  for (;;) {
    const unsigned long long item = wave_uniform(atomicAdd(Q.ctr, one) - Q.base);
    if (item >= total) break;
    const int s = (int)(item / Q.ntiles);
    const int t = (int)(item % Q.ntiles);
    bool go = true;
    if (s > 0) {
      const uint32_t target = Q.epoch + (uint32_t)s;
      uint32_t spins = 0;
      for (;;) {
        const uint32_t p = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(Q.progress + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if ((int32_t)(p - target) >= 0) break;
        if (++spins > SPIN_LIMIT) {
          atomicOr(Q.error, 1);
          go = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      // One acquire after the wait.  An acquire per poll would invalidate
      // the caches (L2 included on this multi-die device) on every iteration,
      // costing every wavefront on the die its cached planet rows.
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int s_begin = s * Q.sub_steps;
    const int s_end = min(Q.nsteps, s_begin + Q.sub_steps);
    if (go && s_begin < s_end) {       // the last sub-chunks of a short chunk may be empty
      const int i = t * 64 + lane;
      advance<NP, KIT, DEPTH, UNIV, true>(w, out, rows, A, i, i < n, s_begin, s_end,
                                          (KargPtr)__builtin_amdgcn_kernarg_segment_ptr());
    }
    // publish completion; the release orders every store of this item
    __hip_atomic_store(Q.progress + t, Q.epoch + (uint32_t)s + 1u, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------- many systems
// Item (s, t) of the batched queue: tile t (64 particles of one system, so the
// planet row stays wave-uniform) through sub-chunk s; the tile's system picks
// the planet count, constants, time step and table rows.
template <int NP>
TPM_DEV void batch_item(const SysDev& S, Work w, Out out, const double* __restrict__ ring,
                        const BatchQueueArgs& Q, const TileDesc& T, int s_begin, int s_end,
                        int lane) {
  ChunkArgs<NP> A;
#pragma unroll
  for (int j = 0; j < (NP > 0 ? NP : 1); ++j) {
    A.P.mu[j] = NP > 0 ? S.mu[j] : 0.0;
    A.P.rcrit2[j] = NP > 0 ? S.rcrit2[j] : 0.0;
  }
  A.K = S.K;
  A.rmax2 = S.rmax2;
  A.ftol = S.ftol;
  A.dt = S.dt;
  A.kiters = S.kiters;
  A.nsteps = Q.nsteps;
  A.step0 = Q.step0;
  A.handoff = 0;
  const double* rows = ring + S.ring_off + (int64_t)Q.slot * Q.slot_rows * (3 * NP + 3);
  const int i = T.first + lane;
  const bool valid = lane < T.count;
  if (S.kiters == 5)
    advance<NP, 5, 0>(w, out, rows, A, i, valid, s_begin, s_end);
  else
    advance<NP, 0, 0>(w, out, rows, A, i, valid, s_begin, s_end);
}

__global__ void __launch_bounds__(256)
particle_batch_queue(const SysDev* __restrict__ sys, const TileDesc* __restrict__ tiles, Work w,
                     Out out, const double* __restrict__ ring, BatchQueueArgs Q) {
  const int lane = threadIdx.x & 63;
  // the tile count of a run that compacts lives on the device (batch_tiles)
  const int ntiles = Q.ntiles_dev ? *Q.ntiles_dev : Q.ntiles;
  const unsigned long long total = (unsigned long long)ntiles * Q.nsub;
  const unsigned long long one = lane == 0 ? 1ull : 0ull;
  for (;;) {
    const unsigned long long item = wave_uniform(atomicAdd(Q.ctr, one) - Q.base);
    if (item >= total) break;
    const int s = (int)(item / ntiles);
    const int t = (int)(item % ntiles);
    bool go = true;
    if (s > 0) {
      const uint32_t target = Q.epoch + (uint32_t)s;
      uint32_t spins = 0;
      for (;;) {
        const uint32_t p = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(Q.progress + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if ((int32_t)(p - target) >= 0) break;
        if (++spins > SPIN_LIMIT) {
          atomicOr(Q.error, 1);
          go = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      // One acquire after the wait.  An acquire per poll would invalidate
      // the caches (L2 included on this multi-die device) on every iteration,
      // costing every wavefront on the die its cached planet rows.
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int s_begin = s * Q.sub_steps;
    const int s_end = min(Q.nsteps, s_begin + Q.sub_steps);
    if (go && s_begin < s_end) {
      const TileDesc T = tiles[t];
      const SysDev& S = sys[T.sys];
      switch (S.np) {
        case 0: batch_item<0>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 1: batch_item<1>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 2: batch_item<2>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 3: batch_item<3>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 4: batch_item<4>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 5: batch_item<5>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 6: batch_item<6>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        case 7: batch_item<7>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
        default: batch_item<8>(S, w, out, ring, Q, T, s_begin, s_end, lane); break;
      }
    }
    __hip_atomic_store(Q.progress + t, Q.epoch + (uint32_t)s + 1u, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_particle_batch(const SysDev* sys, const TileDesc* tiles, Work w, Out out,
                                 const double* ring, const BatchQueueArgs& Q, int workers,
                                 int block, hipStream_t st) {
  if (Q.ntiles <= 0) return hipSuccess;
  const int wpb = block / 64;
  const int nblocks = (workers + wpb - 1) / wpb;
  hipLaunchKernelGGL(particle_batch_queue, dim3(nblocks), dim3(block), 0, st, sys, tiles, w, out,
                     ring, Q);
  return hipGetLastError();
}

// ---- compaction inside a batched run (captured in its graph)
// After a stable partition of the whole working set (launch_compact), each
// system's active particles are still contiguous and in order, so the tiles
// are rebuilt from each system's range [start, end) in the new working set:
// batch_bounds finds the ranges from the slots' systems, batch_tiles lays the
// systems' tiles out in the queue's order (most planets first) and stores the
// new tile count for the next particle launch.
__global__ void __launch_bounds__(256) batch_bounds_clear(int nsys, int32_t* start, int32_t* end) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) { start[s] = 0; end[s] = 0; }
}

__global__ void __launch_bounds__(256)
batch_bounds(const int32_t* __restrict__ slot, const int32_t* __restrict__ d_nactive,
             const int32_t* __restrict__ psys, int32_t* __restrict__ start,
             int32_t* __restrict__ end) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = *d_nactive;
  if (i >= n) return;
  const int s = psys[slot[i]];
  if (i == 0 || psys[slot[i - 1]] != s) start[s] = i;
  if (i == n - 1 || psys[slot[i + 1]] != s) end[s] = i + 1;
}

__global__ void __launch_bounds__(1024)
batch_tiles(const int32_t* __restrict__ sorder, int nsys, const int32_t* __restrict__ start,
            const int32_t* __restrict__ end, TileDesc* __restrict__ tiles,
            int32_t* __restrict__ ntiles_dev) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nsys; base += 1024) {
    const int k = base + threadIdx.x;
    const int s = k < nsys ? sorder[k] : 0;
    const int cnt = k < nsys ? end[s] - start[s] : 0;
    const int nt = (cnt + 63) / 64;
    buf[threadIdx.x] = nt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    const int first = carry + buf[threadIdx.x] - nt;
    for (int j = 0; j < nt; ++j)
      tiles[first + j] = TileDesc{s, start[s] + 64 * j, min(64, cnt - 64 * j), 0};
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ntiles_dev = carry;
}

__global__ void __launch_bounds__(64) queue_reset(unsigned long long* ctr) {
  if (threadIdx.x == 0) *ctr = 0ull;
}

hipError_t launch_batch_retile(Work w, const int32_t* d_nactive, int n_upper, const int32_t* psys,
                               const int32_t* sorder, int nsys, int32_t* start, int32_t* end,
                               TileDesc* tiles, int32_t* ntiles_dev, hipStream_t st) {
  hipLaunchKernelGGL(batch_bounds_clear, dim3((nsys + 255) / 256), dim3(256), 0, st, nsys, start,
                     end);
  if (n_upper > 0)
    hipLaunchKernelGGL(batch_bounds, dim3((n_upper + 255) / 256), dim3(256), 0, st, w.slot,
                       d_nactive, psys, start, end);
  hipLaunchKernelGGL(batch_tiles, dim3(1), dim3(1024), 0, st, sorder, nsys, start, end, tiles,
                     ntiles_dev);
  return hipGetLastError();
}

hipError_t launch_queue_reset(unsigned long long* ctr, hipStream_t st) {
  hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, st, ctr);
  return hipGetLastError();
}

template <int NP>
static hipError_t launch_np(const SysConst& S, Work w, const int32_t* d_nactive, int grid_n,
                            Out out, const double* rows, int nsteps, double dt, int64_t step0,
                            const QueueLaunch& QL, hipStream_t st) {
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
  A.handoff = S.handoff;
  QueueArgs Q;
  Q.ctr = QL.ctr;
  Q.base = QL.base;
  Q.progress = QL.progress;
  Q.epoch = QL.epoch;
  Q.ntiles = (grid_n + 63) / 64;
  Q.nsub = QL.nsub;
  Q.sub_steps = (nsteps + QL.nsub - 1) / QL.nsub;
  Q.nsteps = nsteps;
  Q.error = QL.error;
  if (Q.ntiles <= 0) return hipSuccess;
  const int waves_per_block = QL.block / 64;
  const int nblocks = (QL.workers + waves_per_block - 1) / waves_per_block;
#define TPM_PQ(KIT, UNIV, DEPTH)                                                              \
  hipLaunchKernelGGL((particle_queue<NP, KIT, UNIV, DEPTH>), dim3(nblocks), dim3(QL.block), 0, st, \
                     w, d_nactive, out, rows, A, Q)
  if (QL.deep) {
    if (S.kiters == 5) {
      if (S.universal) TPM_PQ(5, true, 3);
      else TPM_PQ(5, false, 3);
    } else {
      if (S.universal) TPM_PQ(0, true, 3);
      else TPM_PQ(0, false, 3);
    }
  } else {
    if (S.kiters == 5) {
      if (S.universal) TPM_PQ(5, true, 1);
      else TPM_PQ(5, false, 1);
    } else {
      if (S.universal) TPM_PQ(0, true, 1);
      else TPM_PQ(0, false, 1);
    }
  }
#undef TPM_PQ
  return hipGetLastError();
}

hipError_t launch_particle_chunk(const SysConst& S, Work w, const int32_t* d_nactive, int grid_n,
                                 Out out, const double* rows, int nsteps, double dt, int64_t step0,
                                 const QueueLaunch& QL, hipStream_t st) {
  switch (S.np) {
    case 0: return launch_np<0>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 1: return launch_np<1>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 2: return launch_np<2>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 3: return launch_np<3>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 4: return launch_np<4>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 5: return launch_np<5>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 6: return launch_np<6>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 7: return launch_np<7>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    case 8: return launch_np<8>(S, w, d_nactive, grid_n, out, rows, nsteps, dt, step0, QL, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- ephemeris
// The planet map is a serial chain in time, so this kernel is written for
// latency: one wavefront, lane b (1..NP) holds Jacobi body b, lane 0 the
// central body.  Values every lane needs are broadcast with v_readlane into
// scalar registers (no LDS round trip), and everything per step is branch-free
// except the wave-uniform Newton loop of the planets' Kepler drifts.

// Value of v on lane `src` (a compile-time constant), returned wave-uniform
// in an SGPR pair.
TPM_DEV double bcast(double v, int src) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Value of v on lane SRC (below 16) on every lane of each row of 16, by a DPP
// row broadcast (row_newbcast) into a VGPR.  The planet map's bodies sit in
// lanes 0..8, and its other lanes' values are never used: lanes 16..63 then
// carry garbage (NaN included), which every wave-wide test of the planet map
// masks by the lane's idle flag.
template <int SRC>
TPM_DEV double bcast_row(double v) {
  static_assert(SRC >= 0 && SRC < 16, "row broadcast source");
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x150 + SRC, 0xF,
                                                             0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32),
                                                             0x150 + SRC, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The planet map's broadcast of lane src's value.  The single-system map (a
// lone wavefront) reads it into SGPRs, since its FMAs run faster with a scalar
// operand; the many-system map, one wavefront per system, broadcasts it in
// VGPRs, which frees the SGPRs it otherwise spills (3% faster there).
template <bool ROWB>
TPM_DEV double eph_bcast(double v, int src) {
  if (!ROWB) return bcast(v, src);
  switch (src) {
    case 0: return bcast_row<0>(v);
    case 1: return bcast_row<1>(v);
    case 2: return bcast_row<2>(v);
    case 3: return bcast_row<3>(v);
    case 4: return bcast_row<4>(v);
    case 5: return bcast_row<5>(v);
    case 6: return bcast_row<6>(v);
    case 7: return bcast_row<7>(v);
    default: return bcast_row<8>(v);
  }
}

// Heliocentric positions of bodies 0..NP (body 0 at the origin) from the
// Jacobi positions held by lanes 1..NP.  The barycentre of bodies 0..b is
// R_b = R_{b-1} + (mu_b/eta_b) r'_b, so
//   r_b = r'_b + R_{b-1} = r'_b + sum_{k<b} (mu_k/eta_k) r'_k:
// the broadcasts are independent and the chain is one FMA per body.  The
// results are wave-uniform.
template <int NP>
TPM_DEV void helio_all(const EphConst& E, double jx, double jy, double jz,
                       double (&hx)[NP + 1], double (&hy)[NP + 1], double (&hz)[NP + 1]) {
  double Rx = 0.0, Ry = 0.0, Rz = 0.0;
  hx[0] = 0.0; hy[0] = 0.0; hz[0] = 0.0;
#pragma unroll
  for (int b = 1; b <= NP; ++b) {
    const double px = bcast(jx, b), py = bcast(jy, b), pz = bcast(jz, b);
    hx[b] = px + Rx; hy[b] = py + Ry; hz[b] = pz + Rz;
    Rx = fma_(E.cj[b], px, Rx);
    Ry = fma_(E.cj[b], py, Ry);
    Rz = fma_(E.cj[b], pz, Rz);
  }
}

// Per-lane constants of the planet map.
struct EphLane {
  int lane;
  bool body;
  double mup, ie_prev;            // mu'_b, 1/eta_{b-1} (0 on lanes that hold no body)
  double kc;                      // coefficient of the kick's Kepler term (see eph_accel)
  double cw;                      // weight of the central term in the lane's own kick
  double nb;                      // 0 on body lanes, 1 elsewhere (keeps an rsqrt finite)
  double c15;                     // 1.5 (held in a VGPR by the single-system map)
  KepConst K;                     // Kepler constant mu'_b for the drift
};

// Per-lane weights that turn the lane-dependent parts of a step into plain
// FMAs (no selects on the lane index inside the step loop).
template <int NP>
struct EphW {
  double cjv[NP + 1];    // mu_k/eta_k on every lane (see eph_weights)
  double wr[NP + 1];     // mu_k/eta_k for 1 <= k < lane, else 0 (own heliocentric position)
  double wa[NP + 1];     // mu_k for k < lane, else 0 (sum_{k<b} mu_k a_k)
  double mul[NP + 1];    // mu_l, 0 for the lane's own body
  double self[NP + 1];   // 1 for the lane's own body, else 0
  double hill2[NP + 1];  // squared mutual Hill radius with body j > lane, else 0
};

// HOLD: the constants that meet a broadcast in one instruction are held in
// VGPRs (the single-system map, whose broadcasts are scalar); the many-system
// map broadcasts into VGPRs and keeps them as they are.
template <int NP, bool HOLD>
TPM_DEV EphW<NP> eph_weights(const EphConst& E, int lane) {
  EphW<NP> W;
#pragma unroll
  for (int k = 0; k <= NP; ++k) {
    W.cjv[k] = HOLD ? vgpr_held(E.cj[k]) : E.cj[k];
    W.wr[k] = (k >= 1 && k < lane) ? E.cj[k] : 0.0;
    W.wa[k] = (k < lane) ? E.mu[k] : 0.0;
    W.mul[k] = (k == lane) ? 0.0 : E.mu[k];
    W.self[k] = (k == lane) ? 1.0 : 0.0;
    W.hill2[k] = 0.0;
  }
#pragma unroll
  for (int b = 1; b <= NP; ++b)
#pragma unroll
    for (int j = b + 1; j <= NP; ++j)
      if (lane == b) W.hill2[j] = E.hill2[b][j];
  return W;
}

// The lane's own heliocentric position r'_b + R_{b-1} from the broadcast
// Jacobi positions (the same bits as helio_all's entry for body b; 0 on lane
// 0).
template <int NP>
TPM_DEV void own_helio(const EphW<NP>& W, double jx, double jy, double jz,
                       const double (&px)[NP + 1], const double (&py)[NP + 1],
                       const double (&pz)[NP + 1], double& ox, double& oy, double& oz) {
  double Rx = 0.0, Ry = 0.0, Rz = 0.0;
#pragma unroll
  for (int k = 1; k <= NP; ++k) {
    Rx = fma_(W.wr[k], px[k], Rx);
    Ry = fma_(W.wr[k], py[k], Ry);
    Rz = fma_(W.wr[k], pz[k], Rz);
  }
  ox = jx + Rx; oy = jy + Ry; oz = jz + Rz;
}

// Heliocentric positions of all bodies and the lane's own one, from the Jacobi
// positions held by lanes 1..NP (see helio_all).
template <int NP, bool ROWB>
TPM_DEV void helio_step(const EphConst& E, const EphW<NP>& W, double jx, double jy, double jz,
                        double (&hx)[NP + 1], double (&hy)[NP + 1], double (&hz)[NP + 1],
                        double& ox, double& oy, double& oz) {
  double px[NP + 1], py[NP + 1], pz[NP + 1];
  double Rx = 0.0, Ry = 0.0, Rz = 0.0;
  hx[0] = 0.0; hy[0] = 0.0; hz[0] = 0.0;
  px[0] = 0.0; py[0] = 0.0; pz[0] = 0.0;
#pragma unroll
  for (int b = 1; b <= NP; ++b) {
    px[b] = eph_bcast<ROWB>(jx, b); py[b] = eph_bcast<ROWB>(jy, b); pz[b] = eph_bcast<ROWB>(jz, b);
    hx[b] = px[b] + Rx; hy[b] = py[b] + Ry; hz[b] = pz[b] + Rz;
    Rx = fma_(W.cjv[b], px[b], Rx);
    Ry = fma_(W.cjv[b], py[b], Ry);
    Rz = fma_(W.cjv[b], pz[b], Rz);
  }
  own_helio<NP>(W, jx, jy, jz, px, py, pz, ox, oy, oz);
}

// Interaction acceleration of the lane's Jacobi body (lanes 1..NP):
//   a'_b = a_b - (sum_{k<b} mu_k a_k)/eta_{b-1} + mu'_b r'_b/|r'_b|^3,
// with a_k the Newtonian acceleration of body k; lane 0 gets a_0 (h0 = -a_0).
// (ox, oy, oz) is the lane's own heliocentric position.  For the innermost
// body the heliocentric and Jacobi vectors are the same (bit for bit), so its
// central term -mu_0 r/|r|^3 and the Kepler term combine into
// (mu'_1 - mu_0) r/|r|^3: kc holds that difference (exact in floating point,
// the two coefficients being within a factor two) and cw = 0 drops the
// central term from the lane's own sum.  The two terms would otherwise cancel
// to about mu_1/mu_0 of their size and amplify their rounding by mu_0/mu_1.
// The broadcast a_1 keeps its central term.
template <int NP, bool ROWB>
TPM_DEV void eph_accel(const EphConst& E, const EphLane& L, const EphW<NP>& W, double jx,
                       double jy, double jz, const double (&hx)[NP + 1],
                       const double (&hy)[NP + 1], const double (&hz)[NP + 1], double ox,
                       double oy, double oz, double& ax, double& ay, double& az) {
  // the planets' pulls (l >= 1), then the central body's (l = 0, at the origin)
  double px = 0.0, py = 0.0, pz = 0.0;
#pragma unroll
  for (int l = 1; l <= NP; ++l) {
    double dx = ox - hx[l], dy = oy - hy[l], dz = oz - hz[l];
    double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
    double k = mul_rsqrt3(W.mul[l], d2 + W.self[l], L.c15);
    px = fma_(-k, dx, px);
    py = fma_(-k, dy, py);
    pz = fma_(-k, dz, pz);
  }
  const double k0 = mul_rsqrt3(W.mul[0], fma_(ox, ox, fma_(oy, oy, oz * oz)) + W.self[0], L.c15);
  const double nx = fma_(-k0, ox, px), ny = fma_(-k0, oy, py), nz = fma_(-k0, oz, pz);
  // sum_{k<b} mu_k a_k from the broadcast Newtonian accelerations
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    sx = fma_(W.wa[k], eph_bcast<ROWB>(nx, k), sx);
    sy = fma_(W.wa[k], eph_bcast<ROWB>(ny, k), sy);
    sz = fma_(W.wa[k], eph_bcast<ROWB>(nz, k), sz);
  }
  double r2 = fma_(jx, jx, fma_(jy, jy, jz * jz));
  double kk = mul_rsqrt3(L.kc, r2 + L.nb, L.c15);
  const double kw = k0 * L.cw;
  // lane 0: jx = ie_prev = 0, so a = n
  ax = fma_(kk, jx, fma_(-sx, L.ie_prev, fma_(-kw, ox, px)));
  ay = fma_(kk, jy, fma_(-sy, L.ie_prev, fma_(-kw, oy, py)));
  az = fma_(kk, jz, fma_(-sz, L.ie_prev, fma_(-kw, oz, pz)));
}

// Any pair (lane, j > lane) closer than their mutual Hill radius.
template <int NP>
TPM_DEV bool hill_violation(const EphW<NP>& W, double ox, double oy, double oz,
                            const double (&hx)[NP + 1], const double (&hy)[NP + 1],
                            const double (&hz)[NP + 1]) {
  bool bad = false;
#pragma unroll
  for (int j = 2; j <= NP; ++j) {
    double dx = ox - hx[j], dy = oy - hy[j], dz = oz - hz[j];
    double d2 = fma_(dx, dx, fma_(dy, dy, dz * dz));
    bad = bad || (d2 < W.hill2[j]);
  }
  return bad;
}

// The planet map's kernels keep the two-address FP64 FMA (v_fmac_f64), which
// the library's build otherwise turns off: its lone wavefront runs faster with
// the shorter encoding, the particle kernels without the copies it costs.
// (A device-code attribute: the host pass of the same source does not know it.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TPM_PLANET_KERNEL __attribute__((target("fmacf64-inst")))
#else
#define TPM_PLANET_KERNEL
#endif

// Heliocentric velocities of the planets (internal order, [NP][3]) from the
// Jacobi velocities held by lanes 1..NP: the same linear map as the
// positions'.  Wave-uniform call.
template <int NP, bool ROWB>
TPM_DEV void write_helio_velocities(const EphConst& E, const EphW<NP>& W, bool body, int lane,
                                    double wx, double wy, double wz, double* __restrict__ out) {
  double hx[NP + 1], hy[NP + 1], hz[NP + 1];
  double ox, oy, oz;
  helio_step<NP, ROWB>(E, W, wx, wy, wz, hx, hy, hz, ox, oy, oz);
  if (body) {
    out[3 * (lane - 1) + 0] = ox;
    out[3 * (lane - 1) + 1] = oy;
    out[3 * (lane - 1) + 2] = oz;
  }
}

// One step of the planet map (sec. 2.2, planet integration: kick, Jacobi
// drift, kick), from the Jacobi state (j, w) and the interaction acceleration
// a at it; writes table row `row` (this lane's entry).  key1 = 2t for step
// t of the launch: the general form (FAST false) keeps the first event as a
// key ordered in time (see ephemeris_body); the fast form returns instead
// whether the lane would have taken another path than its own (the general
// drift's branches), or, with events on, met an event at all.
template <int NP, bool ROWB, bool FAST, bool VEL>
TPM_DEV bool eph_step(const EphConst& E, const EphLane& L, const EphW<NP>& W, double h, double dt,
                      double& jx, double& jy, double& jz, double& wx, double& wy, double& wz,
                      double& ax, double& ay, double& az, bool writer, double rsign,
                      double* __restrict__ row, double* __restrict__ vrow, uint32_t key1,
                      bool events, uint32_t& first_ev) {
  double hx[NP + 1], hy[NP + 1], hz[NP + 1];
  double ox, oy, oz;
  wx = fma_(h, ax, wx); wy = fma_(h, ay, wy); wz = fma_(h, az, wz);
  bool bad;
  const bool bound = drift_converged_t<FAST>(L.K, dt, L.body, jx, jy, jz, wx, wy, wz, bad);
  if (FAST) bad = bad | (events & L.body & !bound);
  else first_ev = __builtin_elementwise_min(first_ev, (L.body && !bound) ? key1 : UINT32_MAX);
  helio_step<NP, ROWB>(E, W, jx, jy, jz, hx, hy, hz, ox, oy, oz);
  eph_accel<NP, ROWB>(E, L, W, jx, jy, jz, hx, hy, hz, ox, oy, oz, ax, ay, az);
  wx = fma_(h, ax, wx); wy = fma_(h, ay, wy); wz = fma_(h, az, wz);
  if (writer) {
    row[0] = fma_(rsign, ax, ox);
    row[1] = fma_(rsign, ay, oy);
    row[2] = fma_(rsign, az, oz);
  }
  if (NP > 1) {
    const bool close = hill_violation<NP>(W, ox, oy, oz, hx, hy, hz);
    if (FAST) bad = bad | (events & close);
    else first_ev = __builtin_elementwise_min(first_ev, close ? key1 + 1u : UINT32_MAX);
  }
  if (VEL) write_helio_velocities<NP, ROWB>(E, W, L.body, L.lane, wx, wy, wz, vrow);
  return bad;
}

// Steps of one fast block (see ephemeris_body).
constexpr int EPH_BLOCK = 64;

// vside (may be null): receives the planets' heliocentric velocities at the
// chunk's first and last rows, [2][NP][3] (for the sampled diagnostics).
// VEL: vrows receives them at every row, [nsteps+1][NP][3] (for the
// encounter integrator).
template <int NP, bool ROWB, bool VEL = false>
TPM_DEV void ephemeris_body(const EphConst& E, double* __restrict__ rj, double* __restrict__ vj,
                            double* __restrict__ rows, int nsteps, double dt, int64_t step0,
                            int64_t* __restrict__ flag, double* __restrict__ vside = nullptr,
                            double* __restrict__ vrows = nullptr) {
  constexpr int ROW = 3 * NP + 3;
  // This wave is a serial chain that shares its SIMD with particle waves:
  // let it issue first.
  __builtin_amdgcn_s_setprio(3);
  EphLane L;
  L.lane = threadIdx.x;
  L.body = L.lane >= 1 && L.lane <= NP;
  L.mup = 1.0; L.ie_prev = 0.0; L.nb = L.body ? 0.0 : 1.0;
#pragma unroll
  for (int b = 1; b <= NP; ++b)
    if (L.lane == b) { L.mup = E.mup[b]; L.ie_prev = E.inv_eta[b - 1]; }
  L.kc = L.mup;
  L.cw = 1.0;
  L.c15 = ROWB ? 1.5 : vgpr_held(1.5);
  if (NP >= 1 && L.lane == 1) {
    L.kc = E.mup[1] - E.mu[0];
    L.cw = 0.0;
  }
  const EphW<NP> W = eph_weights<NP, !ROWB>(E, L.lane);
  {
    double smu, rsmu;
    sqrt_rsqrt(L.mup, smu, rsmu);
    L.K = KepConst{L.mup, rcp(L.mup), smu, rsmu};
  }
  double jx = 0, jy = 0, jz = 0, wx = 0, wy = 0, wz = 0;
  if (L.body) {
    jx = rj[3 * (L.lane - 1) + 0]; jy = rj[3 * (L.lane - 1) + 1]; jz = rj[3 * (L.lane - 1) + 2];
    wx = vj[3 * (L.lane - 1) + 0]; wy = vj[3 * (L.lane - 1) + 1]; wz = vj[3 * (L.lane - 1) + 2];
  }
  double hx[NP + 1], hy[NP + 1], hz[NP + 1];
  double ox, oy, oz, ax, ay, az;
  helio_step<NP, ROWB>(E, W, jx, jy, jz, hx, hy, hz, ox, oy, oz);
  eph_accel<NP, ROWB>(E, L, W, jx, jy, jz, hx, hy, hz, ox, oy, oz, ax, ay, az);
  // Row entries: lane b writes planet b's heliocentric position, lane 0 (the
  // central body, whose own position is the origin) writes h0 = -a_0, both as
  // fma(rsign, a, o) with rsign = 0 on body lanes and -1 on lane 0.
  const bool writer = L.lane <= NP;
  const int roff = L.body ? 3 * (L.lane - 1) : 3 * NP;
  const double rsign = L.body ? 0.0 : -1.0;
  // row 0: the current state
  if (writer) {
    rows[roff + 0] = fma_(rsign, ax, ox);
    rows[roff + 1] = fma_(rsign, ay, oy);
    rows[roff + 2] = fma_(rsign, az, oz);
  }
  const double h = 0.5 * dt;
  // Per lane, the first event as a key ordered in time, counted from step0: a
  // close pair seen at step step0 + t has key 2t+1; an orbit found unbound
  // while drifting from step0 + t - 1 to step0 + t has key 2t, so it wins a tie
  // with a close pair at that step (it is found first).  Keys grow with t, so
  // the first event is the smallest key.
  uint32_t first_ev = UINT32_MAX;
  if (NP > 1 && hill_violation<NP>(W, ox, oy, oz, hx, hy, hz)) first_ev = 1u;
  if (vside) write_helio_velocities<NP, ROWB>(E, W, L.body, L.lane, wx, wy, wz, vside);
  if (VEL) write_helio_velocities<NP, ROWB>(E, W, L.body, L.lane, wx, wy, wz, vrows);
  // Blocks of EPH_BLOCK steps.  Giant planets on near-circular orbits take
  // the general drift's short sin/cos path and leave its Newton loop after
  // two steps every time, and meet no event; the fast form runs exactly that,
  // with none of the general form's wave-uniform branches, and only notes on
  // each lane whether the general form would have done otherwise.  A block in
  // which any lane did is restored from its start and run again in the
  // general form, as is the rest of the launch.  Either way the rows and the
  // state are the general form's bit for bit.  Once the run's first event is
  // on record (*flag != -1) later events cannot change it and no longer stop
  // the fast form.  (The many-system map keeps the general form: its
  // wavefronts share SIMDs with the particles, which hide its branches.)
  const bool events = *flag == -1;
  bool fast = !ROWB;
  for (int s0 = 0; s0 < nsteps; s0 += EPH_BLOCK) {
    const int nb = nsteps - s0 < EPH_BLOCK ? nsteps - s0 : EPH_BLOCK;
    if (!ROWB && fast) {
      const double sjx = jx, sjy = jy, sjz = jz, swx = wx, swy = wy, swz = wz;
      const double sax = ax, say = ay, saz = az;
      bool bad = false;
      for (int t = 0; t < nb; ++t) {
        const int s = s0 + t;
        bad = bad | eph_step<NP, ROWB, true, VEL>(
                        E, L, W, h, dt, jx, jy, jz, wx, wy, wz, ax, ay, az, writer, rsign,
                        rows + (size_t)(s + 1) * ROW + roff,
                        VEL ? vrows + (size_t)(s + 1) * 3 * NP : nullptr, 2u * (uint32_t)(s + 1),
                        events, first_ev);
      }
      if (wave_all(!bad)) continue;
      jx = sjx; jy = sjy; jz = sjz; wx = swx; wy = swy; wz = swz;
      ax = sax; ay = say; az = saz;
      fast = false;
    }
    for (int t = 0; t < nb; ++t) {
      const int s = s0 + t;
      eph_step<NP, ROWB, false, VEL>(E, L, W, h, dt, jx, jy, jz, wx, wy, wz, ax, ay, az, writer,
                                     rsign, rows + (size_t)(s + 1) * ROW + roff,
                                     VEL ? vrows + (size_t)(s + 1) * 3 * NP : nullptr,
                                     2u * (uint32_t)(s + 1), events, first_ev);
    }
  }
  if (vside) write_helio_velocities<NP, ROWB>(E, W, L.body, L.lane, wx, wy, wz, vside + 3 * NP);
  if (L.body) {
    rj[3 * (L.lane - 1) + 0] = jx; rj[3 * (L.lane - 1) + 1] = jy; rj[3 * (L.lane - 1) + 2] = jz;
    vj[3 * (L.lane - 1) + 0] = wx; vj[3 * (L.lane - 1) + 1] = wy; vj[3 * (L.lane - 1) + 2] = wz;
  }
  // earliest event over the wavefront: unbound -> -2, a close pair -> its step
  uint32_t ev = first_ev;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(ev, off, 64);
    ev = o < ev ? o : ev;
  }
  if (L.lane == 0 && *flag == -1 && ev != UINT32_MAX)
    *flag = (ev & 1u) ? step0 + (int64_t)(ev >> 1) : -2;
}

template <int NP, bool VEL>
__global__ void __launch_bounds__(64) TPM_PLANET_KERNEL
ephemeris_chunk(EphConst E, double* __restrict__ rj, double* __restrict__ vj,
                double* __restrict__ rows, int nsteps, double dt, int64_t step0,
                int64_t* __restrict__ flag, double* __restrict__ vside, double* __restrict__ vrows) {
  ephemeris_body<NP, false, VEL>(E, rj, vj, rows, nsteps, dt, step0, flag, vside, vrows);
}

// Many systems at once: workgroup b runs system b (its constants, Jacobi
// state, table rows and flag are found through the per-system arrays).
__global__ void __launch_bounds__(64) TPM_PLANET_KERNEL
ephemeris_batch(const EphConst* __restrict__ E, double* __restrict__ rj, double* __restrict__ vj,
                double* __restrict__ ring, const int64_t* __restrict__ ring_off, int slot,
                int64_t slot_stride_rows, int nsteps, const double* __restrict__ dt,
                int64_t step0, int64_t* __restrict__ flag) {
  const int b = blockIdx.x;
  const EphConst& e = E[b];
  double* rows = ring + ring_off[b] + (int64_t)slot * slot_stride_rows * (3 * e.np + 3);
  double* r = rj + 3 * MAX_NP * b;
  double* v = vj + 3 * MAX_NP * b;
  switch (e.np) {
    case 1: ephemeris_body<1, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 2: ephemeris_body<2, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 3: ephemeris_body<3, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 4: ephemeris_body<4, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 5: ephemeris_body<5, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 6: ephemeris_body<6, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 7: ephemeris_body<7, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    case 8: ephemeris_body<8, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
    default: ephemeris_body<0, true>(e, r, v, rows, nsteps, dt[b], step0, flag + b); break;
  }
}

// The planet map's event keys count the steps of one launch in 32 bits.
constexpr int MAX_EPH_STEPS = 1 << 30;

hipError_t launch_ephemeris_batch(const EphConst* E, double* rj, double* vj, double* ring,
                                  const int64_t* ring_off, int slot, int64_t slot_stride_rows,
                                  int nsys, int nsteps, const double* dt, int64_t step0,
                                  int64_t* flag, hipStream_t st) {
  if (nsteps < 0 || nsteps > MAX_EPH_STEPS) return hipErrorInvalidValue;
  if (nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(ephemeris_batch, dim3(nsys), dim3(64), 0, st, E, rj, vj, ring, ring_off, slot,
                     slot_stride_rows, nsteps, dt, step0, flag);
  return hipGetLastError();
}

template <int NP>
static hipError_t eph_np(const EphConst& E, double* rj, double* vj, double* rows, int nsteps,
                         double dt, int64_t step0, int64_t* flag, double* vside, double* vrows,
                         hipStream_t st) {
  if (vrows)
    hipLaunchKernelGGL((ephemeris_chunk<NP, true>), dim3(1), dim3(64), 0, st, E, rj, vj, rows,
                       nsteps, dt, step0, flag, vside, vrows);
  else
    hipLaunchKernelGGL((ephemeris_chunk<NP, false>), dim3(1), dim3(64), 0, st, E, rj, vj, rows,
                       nsteps, dt, step0, flag, vside, vrows);
  return hipGetLastError();
}

hipError_t launch_ephemeris_chunk(const EphConst& E, double* rj, double* vj, double* rows,
                                  int nsteps, double dt, int64_t step0, int64_t* flag,
                                  hipStream_t st, double* vside, double* vrows) {
  if (nsteps < 0 || nsteps > MAX_EPH_STEPS) return hipErrorInvalidValue;
  switch (E.np) {
#define TPM_EPH(N) \
    case N: return eph_np<N>(E, rj, vj, rows, nsteps, dt, step0, flag, vside, vrows, st);
    TPM_EPH(0) TPM_EPH(1) TPM_EPH(2) TPM_EPH(3) TPM_EPH(4) TPM_EPH(5) TPM_EPH(6) TPM_EPH(7)
    TPM_EPH(8)
#undef TPM_EPH
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

// Heliocentric -> Jacobi for many systems: workgroup b converts system b's
// planets (arrays [nsys][MAX_NP][3]).
__global__ void __launch_bounds__(64)
helio_to_jacobi_batch(const EphConst* __restrict__ E, const double* __restrict__ h,
                      double* __restrict__ j) {
  const int b = blockIdx.x;
  const EphConst& e = E[b];
  const int lane = threadIdx.x;
  if (lane < 1 || lane > e.np) return;
  const double* hb = h + 3 * MAX_NP * b;
  double* jb = j + 3 * MAX_NP * b;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int k = 1; k < lane; ++k) {
    sx = fma_(e.mu[k], hb[3 * (k - 1) + 0], sx);
    sy = fma_(e.mu[k], hb[3 * (k - 1) + 1], sy);
    sz = fma_(e.mu[k], hb[3 * (k - 1) + 2], sz);
  }
  const double ie = e.inv_eta[lane - 1];
  jb[3 * (lane - 1) + 0] = fma_(-sx, ie, hb[3 * (lane - 1) + 0]);
  jb[3 * (lane - 1) + 1] = fma_(-sy, ie, hb[3 * (lane - 1) + 1]);
  jb[3 * (lane - 1) + 2] = fma_(-sz, ie, hb[3 * (lane - 1) + 2]);
}

hipError_t launch_helio_to_jacobi_batch(const EphConst* E, const double* h, double* j, int nsys,
                                        hipStream_t st) {
  if (nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(helio_to_jacobi_batch, dim3(nsys), dim3(64), 0, st, E, h, j);
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

// Per argument: rsqrt, sqrt (sqrt_rsqrt), rcp, mul_rsqrt3(1, x), mul_rsqrt3_1(1, x).
__global__ void rsqrt_test_kernel(const double* x, double* out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  double sq, rs;
  sqrt_rsqrt(v, sq, rs);
  out[5 * (size_t)i + 0] = rsqrt(v);
  out[5 * (size_t)i + 1] = sq;
  out[5 * (size_t)i + 2] = rcp(v);
  out[5 * (size_t)i + 3] = mul_rsqrt3(1.0, v);
  out[5 * (size_t)i + 4] = mul_rsqrt3_1(1.0, v);
}

hipError_t launch_rsqrt_test(const double* x, double* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rsqrt_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, out, n);
  return hipGetLastError();
}

// mode 0: the fixed-iteration drift; 1: as the particle kernel with the
// universal fallback; 2: the universal-variable drift alone.
__global__ void drift_test_kernel(KepConst K, int kiters, double ftol, const double* in,
                                  double* out, int32_t* ok, int n, double dt, int mode) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = in[6 * i + 0], y = in[6 * i + 1], z = in[6 * i + 2];
  double vx = in[6 * i + 3], vy = in[6 * i + 4], vz = in[6 * i + 5];
  bool g = false;
  if (mode != 2) g = drift_fixed(K, dt, kiters, ftol, x, y, z, vx, vy, vz);
  if (mode != 0 && !g) {
    x = in[6 * i + 0]; y = in[6 * i + 1]; z = in[6 * i + 2];
    vx = in[6 * i + 3]; vy = in[6 * i + 4]; vz = in[6 * i + 5];
    g = drift_universal(K.mu, dt, x, y, z, vx, vy, vz);
  }
  // a refused drift leaves the state as it was
  out[6 * i + 0] = g ? x : in[6 * i + 0]; out[6 * i + 1] = g ? y : in[6 * i + 1];
  out[6 * i + 2] = g ? z : in[6 * i + 2]; out[6 * i + 3] = g ? vx : in[6 * i + 3];
  out[6 * i + 4] = g ? vy : in[6 * i + 4]; out[6 * i + 5] = g ? vz : in[6 * i + 5];
  ok[i] = g ? 1 : 0;
}

hipError_t launch_drift_test(const SysConst& S, const double* rv_in, double* rv_out, int32_t* ok,
                             int n, double dt, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  KepConst K{S.mu0, S.inv_mu0, S.sqrt_mu0, S.inv_sqrt_mu0};
  hipLaunchKernelGGL(drift_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, K, S.kiters,
                     S.ftol, rv_in, rv_out, ok, n, dt, S.universal);
  return hipGetLastError();
}

}  // namespace tpm
