// tpm_integrate_static: one whole run (planets set, particles set, integrated,
// results written) on caller-owned device buffers, with every buffer the
// kernels need beyond the inputs and outputs taken from a fixed device array
// of this library.  It allocates nothing, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).
//
// The array, `scratch`, is a file-scope __device__ array, so each GPU the
// library runs on holds its own copy until the process ends.  Its address on
// a device is taken once, with that device current, by hipGetSymbolAddress;
// host code uses only that address (the array's name in host code is a
// host-side stand-in, not a device address).  Every call on a GPU shares the
// GPU's array: calls that overlap on one GPU race, and each call initialises
// what it uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tpmvs.h"
#include "ad_internal.h"
#include "internal.h"

using namespace tpm;

namespace {

constexpr int64_t S_MAX_N = int64_t(1) << 18;     // particles
constexpr int S_MAX_CHUNK = 8192;                 // steps per chunk
constexpr int64_t S_MAX_TILES = S_MAX_N / 64;
constexpr int64_t S_ROW = 3 * MAX_NP + 3;         // doubles per planet-table row, at most

// Byte layout of the array (every part 256-byte aligned).
constexpr int64_t al(int64_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t OFF_WORK0 = 0;                                   // 6 doubles + 2 ints per particle
constexpr int64_t WORK_BYTES = al(S_MAX_N * 56);
constexpr int64_t OFF_WORK1 = OFF_WORK0 + WORK_BYTES;
constexpr int64_t OFF_RING = OFF_WORK1 + WORK_BYTES;               // one chunk of planet rows
constexpr int64_t RING_BYTES = al((S_MAX_CHUNK + 1) * S_ROW * 8);
constexpr int64_t OFF_PROG = OFF_RING + RING_BYTES;                // per-tile progress
constexpr int64_t PROG_BYTES = al(S_MAX_TILES * 4);
constexpr int64_t OFF_CSCR = OFF_PROG + PROG_BYTES;                // compaction scratch
constexpr int64_t CSCR_BYTES = al((2 * (S_MAX_N / 1024 + 1) + 2) * 4);
constexpr int64_t OFF_PLAN = OFF_CSCR + CSCR_BYTES;                // rj, vj, helio r, v
constexpr int64_t PLAN_BYTES = al(4 * 3 * MAX_NP * 8);
constexpr int64_t OFF_MISC = OFF_PLAN + PLAN_BYTES;                // counters and flags
constexpr int64_t MISC_BYTES = 256;
constexpr int64_t SCRATCH_BYTES = OFF_MISC + MISC_BYTES;
static_assert(SCRATCH_BYTES <= (int64_t(32) << 20), "scratch exceeds 32 MiB");

struct Misc {
  unsigned long long qctr;   // work-queue item counter
  int64_t flag;              // planet event (see tpm_integrate_static)
  int32_t nactive;
  int32_t qerr;              // work-queue error flag
};
static_assert(sizeof(Misc) <= MISC_BYTES, "misc block");

}  // namespace

// about 30 MiB per device
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

// Heliocentric planet state passed by value (no device buffer needed).
struct PlanetsIn {
  double r[3 * MAX_NP];
  double v[3 * MAX_NP];
};

// Initial state of one run: working set 0's slots (caller index) and status
// (all active), the planets' heliocentric state, the progress words of the
// tiles, and the counters and flags.
__global__ void __launch_bounds__(256)
static_setup_kernel(unsigned char* base, PlanetsIn P, int np, int n, int ntiles) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t* slot = reinterpret_cast<int32_t*>(base + OFF_WORK0 + 48 * (int64_t)n);
  if (i < n) {
    slot[i] = i;
    slot[n + i] = 0;      // the status array follows the slots
  }
  if (i < ntiles) reinterpret_cast<uint32_t*>(base + OFF_PROG)[i] = 0u;
  if (i < 3 * np) {
    double* h = reinterpret_cast<double*>(base + OFF_PLAN) + 2 * 3 * MAX_NP;
    h[i] = P.r[i];
    h[3 * MAX_NP + i] = P.v[i];
  }
  if (i == 0) {
    Misc* m = reinterpret_cast<Misc*>(base + OFF_MISC);
    m->qctr = 0ull;
    m->flag = -1;
    m->nactive = n;
    m->qerr = 0;
  }
}

// Copies the planet event and the work-queue error flag to the caller.
__global__ void static_finish_kernel(const unsigned char* base, int64_t* info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const Misc* m = reinterpret_cast<const Misc*>(base + OFF_MISC);
    info[0] = m->flag;
    info[1] = m->qerr;
  }
}

// Work set k of n particles inside the array: x, y, z, vx, vy, vz, slot, status.
Work work_at(unsigned char* base, int k, int n) {
  unsigned char* b = base + (k == 0 ? OFF_WORK0 : OFF_WORK1);
  double* d = reinterpret_cast<double*>(b);
  Work w;
  w.x = d; w.y = d + n; w.z = d + 2 * (int64_t)n;
  w.vx = d + 3 * (int64_t)n; w.vy = d + 4 * (int64_t)n; w.vz = d + 5 * (int64_t)n;
  w.slot = reinterpret_cast<int32_t*>(b + 48 * (int64_t)n);
  w.status = w.slot + n;
  return w;
}

int sfail(int code, const std::string& msg) { return set_error(code, msg.c_str()); }

#define S_HIP(expr)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return sfail(TPM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// The array's address and the compute-unit count of each device, taken once
// per device with that device current.
struct DevEntry {
  unsigned char* base = nullptr;
  int ncu = 0;
};

int device_entry(int dev, DevEntry& out) {
  static std::mutex m;
  static std::vector<DevEntry> table;
  std::lock_guard<std::mutex> g(m);
  if ((int)table.size() <= dev) table.resize(dev + 1);
  DevEntry& e = table[dev];
  if (!e.base) {
    void* p = nullptr;
    S_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    int ncu = 0;
    S_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    e.base = static_cast<unsigned char*>(p);
    e.ncu = ncu;
  }
  out = e;
  return TPM_OK;
}

}  // namespace

extern "C" int tpm_integrate_static(const tpm_options* opt_in, double mu0, int32_t np,
                                    const double* mu, const double* rp, const double* vp,
                                    const double* rcrit, int64_t n, const double* d_r,
                                    const double* d_v, int64_t nsteps, double dt, double* d_r_out,
                                    double* d_v_out, int64_t* d_step, int32_t* d_reason,
                                    int32_t* d_planet, int64_t* d_info, void* stream) {
  // ---- validation (host only; nothing is enqueued on a refusal)
  tpm_options o;
  tpm_default_options(&o);
  if (opt_in) o = *opt_in;
  if (o.kepler_iters <= 0) o.kepler_iters = 5;
  if (o.kepler_iters > 64) return sfail(TPM_EINVAL, "kepler_iters > 64");
  if (o.handoff_substeps != 0)
    return sfail(TPM_EINVAL, "the close-encounter hand-off does not run without allocation");
  if (o.chunk_steps < 0 || o.resync_chunks < 0 || o.block_threads < 0 || o.sub_chunks < 0 ||
      o.waves_per_simd < 0)
    return sfail(TPM_EINVAL, "negative option");
  if (o.chunk_steps == 0) o.chunk_steps = S_MAX_CHUNK;
  if (o.chunk_steps > S_MAX_CHUNK)
    return sfail(TPM_EINVAL, "chunk_steps above the static limit of 8192");
  if (o.resync_chunks == 0) o.resync_chunks = 1;
  if (o.block_threads == 0) o.block_threads = 64;
  if (o.block_threads % 64 || o.block_threads > 256)
    return sfail(TPM_EINVAL, "block_threads must be 64, 128, 192 or 256");
  if (o.sub_chunks == 0) o.sub_chunks = 64;
  if (o.waves_per_simd > 8) return sfail(TPM_EINVAL, "waves_per_simd > 8");
  if (!(o.kepler_ftol > 0.0)) o.kepler_ftol = 1e-13;
  if (!std::isfinite(o.r_escape)) return sfail(TPM_EINVAL, "r_escape not finite");
  if (!(std::isfinite(mu0) && mu0 > 0.0)) return sfail(TPM_EINVAL, "mu0 must be finite and > 0");
  if (np < 0 || np > MAX_NP) return sfail(TPM_EINVAL, "np must be in 0..8");
  if (np > 0 && (!mu || !rp || !vp || !rcrit)) return sfail(TPM_EINVAL, "NULL planet array");
  if (n < 0) return sfail(TPM_EINVAL, "n < 0");
  if (n > S_MAX_N)
    return sfail(TPM_EINVAL, "n = " + std::to_string(n) + " exceeds the static limit of " +
                                 std::to_string(S_MAX_N) + " particles");
  if (n > 0 && (!d_r || !d_v || !d_r_out || !d_v_out || !d_step || !d_reason || !d_planet))
    return sfail(TPM_EINVAL, "NULL particle buffer");
  if (nsteps < 0 || nsteps >= (int64_t(1) << 40)) return sfail(TPM_EINVAL, "nsteps out of range");
  if (!std::isfinite(dt) || dt == 0.0) return sfail(TPM_EINVAL, "dt must be finite and non-zero");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return sfail(TPM_EDEVICE, "no HIP device");
  if (o.device < 0 || o.device >= ndev) return sfail(TPM_EINVAL, "device ordinal out of range");
  // planets: bound orbits, sorted by osculating semi-major axis (Jacobi order)
  double a[MAX_NP] = {0};
  for (int j = 0; j < np; ++j) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(rp[3 * j + k]) || !std::isfinite(vp[3 * j + k]))
        return sfail(TPM_EINVAL, "planet input not finite");
    if (!(std::isfinite(mu[j]) && mu[j] > 0.0)) return sfail(TPM_EINVAL, "planet mu must be > 0");
    if (!(std::isfinite(rcrit[j]) && rcrit[j] >= 0.0)) return sfail(TPM_EINVAL, "r_crit must be >= 0");
    const double rr = std::sqrt(rp[3 * j] * rp[3 * j] + rp[3 * j + 1] * rp[3 * j + 1] +
                                rp[3 * j + 2] * rp[3 * j + 2]);
    const double vv = vp[3 * j] * vp[3 * j] + vp[3 * j + 1] * vp[3 * j + 1] + vp[3 * j + 2] * vp[3 * j + 2];
    const double alpha = 2.0 / rr - vv / (mu0 + mu[j]);
    if (!(rr > 0.0) || !(alpha > 0.0)) return sfail(TPM_EINVAL, "planet orbit not bound");
    a[j] = 1.0 / alpha;
  }
  int perm[MAX_NP];
  std::iota(perm, perm + np, 0);
  std::stable_sort(perm, perm + np, [&](int x, int y) { return a[x] < a[y]; });
  double ms[MAX_NP] = {0}, as[MAX_NP] = {0};
  PlanetsIn P{};
  SysConst S{};
  S.np = np;
  S.mu0 = mu0;
  S.inv_mu0 = 1.0 / mu0;
  S.sqrt_mu0 = std::sqrt(mu0);
  S.inv_sqrt_mu0 = 1.0 / std::sqrt(mu0);
  for (int j = 0; j < np; ++j) {
    const int c = perm[j];
    ms[j] = mu[c];
    as[j] = a[c];
    S.mu[j] = mu[c];
    S.rcrit2[j] = rcrit[c] * rcrit[c];
    for (int k = 0; k < 3; ++k) { P.r[3 * j + k] = rp[3 * c + k]; P.v[3 * j + k] = vp[3 * c + k]; }
  }
  S.rmax2 = o.r_escape > 0 ? o.r_escape * o.r_escape : INFINITY;
  S.kiters = o.kepler_iters;
  S.ftol = o.kepler_ftol;
  // planet-map constants (as the simulation object computes them)
  EphConst E{};
  E.np = np;
  E.mu[0] = mu0;
  E.eta[0] = mu0;
  E.inv_eta[0] = 1.0 / mu0;
  for (int b = 1; b <= np; ++b) {
    E.mu[b] = ms[b - 1];
    E.eta[b] = E.eta[b - 1] + E.mu[b];
    E.inv_eta[b] = 1.0 / E.eta[b];
    E.mup[b] = mu0 * E.eta[b] / E.eta[b - 1];
    E.cj[b] = E.mu[b] / E.eta[b];
  }
  for (int i = 1; i <= np; ++i)
    for (int j = 1; j <= np; ++j) {
      const double rh = std::cbrt((E.mu[i] + E.mu[j]) / (3.0 * mu0)) * 0.5 * (as[i - 1] + as[j - 1]);
      E.hill2[i][j] = rh * rh;
    }

  // ---- device work, all on the caller's stream
  S_HIP(hipSetDevice(o.device));
  DevEntry D;
  {
    int rc = device_entry(o.device, D);
    if (rc) return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  unsigned char* base = D.base;
  const int nn = (int)n;
  const int K = o.chunk_steps;
  const int R = o.resync_chunks;
  const int ntiles = (nn + 63) / 64;
  Misc* misc = reinterpret_cast<Misc*>(base + OFF_MISC);
  double* plan = reinterpret_cast<double*>(base + OFF_PLAN);
  double* rj = plan;
  double* vj = plan + 3 * MAX_NP;
  double* hr = plan + 6 * MAX_NP;
  double* hv = plan + 9 * MAX_NP;
  double* ring = reinterpret_cast<double*>(base + OFF_RING);
  int32_t* cscr = reinterpret_cast<int32_t*>(base + OFF_CSCR);
  {
    const int m = std::max(std::max(nn, ntiles), std::max(3 * np, 1));
    hipLaunchKernelGGL(static_setup_kernel, dim3((m + 255) / 256), dim3(256), 0, st, base, P, np, nn,
                       ntiles);
    S_HIP(hipGetLastError());
  }
  if (np > 0) {
    S_HIP(launch_helio_to_jacobi(E, hr, rj, st));
    S_HIP(launch_helio_to_jacobi(E, hv, vj, st));
  }
  Work w[2] = {work_at(base, 0, nn), work_at(base, 1, nn)};
  S_HIP(launch_aos_to_soa(d_r, d_v, w[0].x, n, st));
  Out out{d_r_out, d_v_out, d_step, d_reason, d_planet};
  int cur = 0;
  unsigned long long q_base = 0;
  uint32_t q_epoch = 0;
  const int64_t nchunks = (nsteps + K - 1) / K;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int ks = (int)std::min<int64_t>(K, nsteps - c * K);
    const int64_t step0 = c * K;
    S_HIP(launch_ephemeris_chunk(E, rj, vj, ring, ks, dt, step0, &misc->flag, st));
    if (nn > 0) {
      QueueLaunch QL;
      QL.ctr = &misc->qctr;
      QL.base = q_base;
      QL.progress = reinterpret_cast<uint32_t*>(base + OFF_PROG);
      QL.epoch = q_epoch;
      const int item = std::max(1, K / std::max(1, o.sub_chunks));
      QL.nsub = std::max(1, std::min(o.sub_chunks, (ks + item - 1) / item));
      const int wps = o.waves_per_simd > 0 ? o.waves_per_simd : auto_waves_per_simd(ntiles, D.ncu);
      QL.workers = std::max(1, std::min(ntiles * QL.nsub, 4 * D.ncu * wps));
      QL.deep = wps == 1;
      QL.workers = std::min(QL.workers, ntiles);
      QL.block = o.block_threads;
      QL.error = &misc->qerr;
      S_HIP(launch_particle_chunk(S, w[cur], &misc->nactive, nn, out, ring, ks, dt, step0, QL, st));
      const int wpb = QL.block / 64;
      const unsigned long long waves = (unsigned long long)((QL.workers + wpb - 1) / wpb) * wpb;
      q_base += (unsigned long long)ntiles * QL.nsub + waves;
      q_epoch += (uint32_t)QL.nsub;
      if (((c + 1) % R == 0) || c == nchunks - 1) {
        S_HIP(launch_compact(w[cur], w[1 - cur], &misc->nactive, nn, cscr, st));
        cur = 1 - cur;
      }
    }
  }
  if (nn > 0) S_HIP(launch_finalize(w[cur], &misc->nactive, nn, out, st));
  if (d_info) {
    hipLaunchKernelGGL(static_finish_kernel, dim3(1), dim3(64), 0, st, base, d_info);
    S_HIP(hipGetLastError());
  }
  return TPM_OK;
}
