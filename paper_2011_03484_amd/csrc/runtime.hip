// Host runtime behind the C ABI of include/tpmvs.h.
//
// One simulation = one device and the device's two HIP streams (default
// priority, shared by every simulation on the device):
//   stream E runs the planet map chunk by chunk into a ring of planet-table
//   slots in HBM; stream P runs the particle kernel over each slot once its
//   rows are written.  The planet map for chunk c+1 thus overlaps the particle
//   work of chunk c (sec. 2.2: the next planetary chunk is prepared while the
//   particles are advanced), with events guarding slot reuse.  Every
//   resync_chunks chunks the working set is compacted (sec. 2.2, resync
//   interval) and its new size read back to shrink the next launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tpmvs.h"
#include "ad_internal.h"
#include "diag_internal.h"
#include "history_internal.h"
#include "internal.h"

using namespace tpm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define TPM_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? TPM_ENOMEM : TPM_EDEVICE,                 \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

// The two streams of a device, created once per process and shared by all
// simulations on that device.  A pair per simulation would let the two
// streams of one simulation land on the same hardware queue once a process
// holds more streams than the runtime has queues, and that serializes the
// planet map behind the particle kernel.  The long pipelined calls
// (integrate, batched integrate) hold the device's lock, so calls from several
// threads on one device run one after another.
struct DeviceStreams {
  std::mutex lock;
  hipStream_t sP = nullptr, sE = nullptr;
  hipStream_t sH = nullptr;   // encounter integrator (close-encounter hand-off), on first use
};

DeviceStreams& device_streams(int dev) {
  static std::mutex m;
  static std::map<int, std::unique_ptr<DeviceStreams>> all;
  std::lock_guard<std::mutex> g(m);
  auto& p = all[dev];
  if (!p) p.reset(new DeviceStreams());
  return *p;
}

// Create the device's stream pair on first use (device already current).
hipError_t ensure_device_streams(DeviceStreams& D) {
  static std::mutex m;
  std::lock_guard<std::mutex> g(m);
  if (D.sP) return hipSuccess;
  hipStream_t a = nullptr, b = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
  if (e != hipSuccess) { (void)hipStreamDestroy(a); return e; }
  D.sP = a;
  D.sE = b;
  return hipSuccess;
}

constexpr int NSLOT = 8;   // planet-table ring slots
constexpr int FIRST_CHUNK_STEPS = 1024;   // longest first chunk of an on-the-fly run
// With the close-encounter hand-off an integrate call keeps all its planet
// rows (and planet velocities); a call that would need more than this (the
// environment variable TPM_HANDOFF_RING_BYTES may set it) is run as several
// calls (survivors of the encounter list rejoin the working set at each one's
// end, which changes no result).
constexpr int64_t HANDOFF_RING_BYTES = int64_t(4) << 30;

int64_t handoff_ring_bytes() {
  const char* e = std::getenv("TPM_HANDOFF_RING_BYTES");
  if (e && *e) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end && *end == '\0' && v > 0) return (int64_t)v;
  }
  return HANDOFF_RING_BYTES;
}
constexpr int NCNT = 8;    // in-flight active-count readbacks

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Device buffers of one call, freed when the holder goes out of scope (also
// on the early error returns of TPM_HIP).
struct DevScope {
  std::vector<void*> held;
  template <class T>
  hipError_t alloc(T*& out, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) {
      held.push_back(q);
      out = static_cast<T*>(q);
    }
    return e;
  }
  ~DevScope() {
    for (void* q : held) (void)hipFree(q);
  }
};

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Planet-map constants of one system from its sorted planets (mu, initial
// osculating semi-major axes).
EphConst make_eph(double mu0, int np, const double* mu, const double* a) {
  EphConst E{};
  E.np = np;
  E.mu[0] = mu0;
  E.eta[0] = mu0;
  E.inv_eta[0] = 1.0 / mu0;
  for (int b = 1; b <= np; ++b) {
    E.mu[b] = mu[b - 1];
    E.eta[b] = E.eta[b - 1] + E.mu[b];
    E.inv_eta[b] = 1.0 / E.eta[b];
    E.mup[b] = mu0 * E.eta[b] / E.eta[b - 1];
    E.cj[b] = E.mu[b] / E.eta[b];
  }
  for (int i = 1; i <= np; ++i)
    for (int j = 1; j <= np; ++j) {
      double rh = std::cbrt((E.mu[i] + E.mu[j]) / (3.0 * mu0)) * 0.5 * (a[i - 1] + a[j - 1]);
      E.hill2[i][j] = rh * rh;
    }
  return E;
}

// Osculating semi-major axes (mu0 + mu_j) of np planets and the order that
// sorts them (the Jacobi order).  Returns false if an orbit is not bound.
bool sort_planets(double mu0, int np, const double* mu, const double* r, const double* v,
                  std::vector<int>& perm, std::vector<double>& a) {
  a.resize(np);
  for (int j = 0; j < np; ++j) {
    double rr = std::sqrt(r[3 * j] * r[3 * j] + r[3 * j + 1] * r[3 * j + 1] + r[3 * j + 2] * r[3 * j + 2]);
    double vv = v[3 * j] * v[3 * j] + v[3 * j + 1] * v[3 * j + 1] + v[3 * j + 2] * v[3 * j + 2];
    double alpha = 2.0 / rr - vv / (mu0 + mu[j]);
    if (!(rr > 0.0) || !(alpha > 0.0)) return false;
    a[j] = 1.0 / alpha;
  }
  perm.resize(np);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return a[x] < a[y]; });
  return true;
}

}  // namespace

int tpm::set_error(int code, const char* msg) { return fail(code, msg); }

struct tpm_sim {
  tpm_options opt{};
  hipStream_t sP = nullptr, sE = nullptr;
  hipEvent_t ev_eph[NSLOT]{}, ev_done[NSLOT]{};
  hipEvent_t t0P = nullptr, t1P = nullptr, t0E = nullptr, t1E = nullptr;
  bool central_set = false, planets_set = false, particles_set = false;
  double mu0 = 0.0;
  int np = 0;
  std::vector<int> perm;                 // internal planet index -> caller index
  std::vector<double> mu_s, rcrit_s;     // internal (sorted) order
  std::vector<double> a_s;               // initial osculating semi-major axes, sorted
  double* d_rj = nullptr;                // Jacobi planet state [np][3]
  double* d_vj = nullptr;
  double* d_tmp = nullptr;               // [4][np][3] scratch for conversions
  int64_t* d_flag = nullptr;
  int64_t n = 0;
  Work work[2]{};
  int cur = 0;
  int32_t* d_nactive = nullptr;
  int32_t* d_scratch = nullptr;
  Out out{};
  int32_t* h_pin = nullptr;             // [0..NCNT) active counts, [16..] scratch
  hipEvent_t ev_cnt[NCNT]{};             // one per in-flight count readback
  int64_t cnt_issued = 0, cnt_seen = 0;  // readbacks issued / consumed
  unsigned long long* d_acc = nullptr;
  int n_active = 0;                      // host copy (upper bound between compactions)
  double* d_ring = nullptr;
  int64_t ring_rows = 0;                 // rows per slot allocated
  int64_t ring_slots = 0;                // slots allocated (NSLOT; with the hand-off, a call's chunks)
  double* d_table = nullptr;             // caller-supplied table (optional)
  int64_t table_rows = 0;
  // planet history (tpm_set_planet_history): t[nrec], r, v [nrec][np][3]
  // in integration order, one device block
  double* d_hist = nullptr;
  int64_t hist_nrec = 0;
  double hist_t0 = 0.0, hist_tmin = 0.0, hist_tmax = 0.0;
  double hist_dt = 0.0;                  // dt of the last integrate (the current time)
  int64_t step = 0;
  int ncu = 0;                           // compute units of the device
  int last_wps = 0;                      // wavefronts per SIMD of the last particle launch
  unsigned long long* d_qctr = nullptr;  // work-queue item counter
  uint32_t* d_progress = nullptr;        // per-tile progress counters
  int32_t* d_qerr = nullptr;             // work-queue error flag
  unsigned long long q_base = 0;         // host copy of the item counter
  uint32_t q_epoch = 0;                  // host copy of the tiles' progress
  tpm_stats stats{};
  // automatic-differentiation context of the last tpm_ad_forward
  struct AD {
    int64_t n = 0, nsteps = 0;
    int ckpt = 0, nseg = 0;
    double dt = 0.0;
    double* table = nullptr;      // [nsteps+1][3np+3]
    double* ckpts = nullptr;      // [nseg+1][6][n]
    double* tape = nullptr;       // [2][ckpt][AD_TAPE_FIELDS][n]: two segments' tapes (see tpm_ad_backward)
    double* work = nullptr;       // [2][6][n]
    int64_t* dstep = nullptr;
    int32_t* reason = nullptr;
    int32_t* planet = nullptr;
    int32_t* treason = nullptr;   // tangent's own removal flags
    size_t cap_table = 0, cap_ckpts = 0, cap_tape = 0, cap_n = 0;
    bool valid = false;
    // ordering events between the caller's stream and the library's streams
    hipEvent_t ev_tab[2]{}, ev_rec[2]{}, ev_rev[2]{}, ev_in = nullptr;
  } ad;
  std::vector<hipEvent_t> kev;           // per-launch timing events (time_kernels)
  // sampled diagnostics and snapshots (tpm_set_diagnostics)
  struct Diag {
    bool on = false;
    int64_t every = 0;
    int nres = 0, ref = -1;                // ref: internal planet index
    int p[2]{}, q[2]{};
    double* emax = nullptr;
    int64_t* estep = nullptr;
    int32_t* flags = nullptr;
    double* lo = nullptr;
    double* hi = nullptr;
    tpm_snapshot_fn snap = nullptr;
    void* user = nullptr;
    char* d_snap = nullptr;                // device snapshot staging, SNAP_BYTES(n)
    char* h_snap[2] = {nullptr, nullptr};  // pinned ring
    hipEvent_t ev_snap[2] = {nullptr, nullptr};
    int64_t last_step = -1;                // last sampled global step
  } diag;
  double* d_vside = nullptr;             // [NSLOT][2][np][3] planet velocities at chunk ends
  // close-encounter hand-off: removal radii (internal order), the encounter
  // list (capacity n), the list's length after each chunk's hand-offs, the
  // planets' velocities per row of every ring slot, and the events ordering
  // the encounter stream
  std::vector<double> rrem_s;
  bool rrem_set = false;
  EncList enc{};
  int32_t* d_snap = nullptr;             // [chunks of the call]
  double* d_vring = nullptr;             // [slots][vring_rows][np][3]
  int64_t vring_rows = 0, vring_slots = 0;
  int vring_np = -1;                     // planets the velocity ring was sized for
  int64_t snap_slots = 0;                // entries of d_snap
  hipEvent_t ev_gath[NSLOT]{}, ev_hdone[NSLOT]{};

  ~tpm_sim() {
    release_handoff();
    for (int k = 0; k < NSLOT; ++k) {
      if (ev_gath[k]) (void)hipEventDestroy(ev_gath[k]);
      if (ev_hdone[k]) (void)hipEventDestroy(ev_hdone[k]);
    }
    release_ad();
    release_diag();
    release_particles();
    release_planets();
    release_ring();
    release_base();
  }
  void release_ad() {
    dfree(ad.table); dfree(ad.ckpts); dfree(ad.tape); dfree(ad.work);
    dfree(ad.dstep); dfree(ad.reason); dfree(ad.planet); dfree(ad.treason);
    for (int k = 0; k < 2; ++k) {
      if (ad.ev_tab[k]) (void)hipEventDestroy(ad.ev_tab[k]);
      if (ad.ev_rec[k]) (void)hipEventDestroy(ad.ev_rec[k]);
      if (ad.ev_rev[k]) (void)hipEventDestroy(ad.ev_rev[k]);
    }
    if (ad.ev_in) (void)hipEventDestroy(ad.ev_in);
    ad = AD{};
  }

  void release_diag() {
    if (sP) (void)hipStreamSynchronize(sP);
    dfree(diag.emax); dfree(diag.estep); dfree(diag.flags); dfree(diag.lo); dfree(diag.hi);
    dfree(diag.d_snap);
    for (int k = 0; k < 2; ++k) {
      if (diag.h_snap[k]) (void)hipHostFree(diag.h_snap[k]);
      if (diag.ev_snap[k]) (void)hipEventDestroy(diag.ev_snap[k]);
    }
    dfree(d_vside);
    diag = Diag{};
  }

  void release_handoff() {
    dfree(enc.x); dfree(enc.y); dfree(enc.z); dfree(enc.vx); dfree(enc.vy); dfree(enc.vz);
    dfree(enc.slot); dfree(enc.status); dfree(enc.step); dfree(enc.m); dfree(enc.Ml);
    dfree(enc.count);
    enc = EncList{};
    dfree(d_snap);
    dfree(d_vring);
    vring_rows = 0;
    vring_slots = 0;
    vring_np = -1;
    snap_slots = 0;
  }
  void release_particles() {
    release_handoff();
    release_diag();
    for (auto& w : work) {
      dfree(w.x); dfree(w.y); dfree(w.z); dfree(w.vx); dfree(w.vy); dfree(w.vz);
      dfree(w.slot); dfree(w.status);
      w = Work{};
    }
    dfree(out.r); dfree(out.v); dfree(out.step); dfree(out.reason); dfree(out.planet);
    out = Out{};
    dfree(d_scratch); d_scratch = nullptr;
    dfree(d_qctr); dfree(d_progress); dfree(d_qerr);
    q_base = 0;
    q_epoch = 0;
    n = 0;
    particles_set = false;
  }
  void release_planets() {
    release_diag();
    dfree(d_rj); dfree(d_vj); dfree(d_tmp); dfree(d_table);
    d_rj = d_vj = d_tmp = d_table = nullptr;
    table_rows = 0;
    release_history();
  }
  void release_history() {
    dfree(d_hist);
    hist_nrec = 0;
  }
  HistDev hist() const {
    HistDev H{};
    H.np = np;
    H.nrec = hist_nrec;
    H.t = d_hist;
    H.r = d_hist + hist_nrec;
    H.v = d_hist + hist_nrec * (1 + 3 * np);
    for (int j = 0; j < np; ++j) H.mu[j] = mu_s[j];
    H.t0 = hist_t0;
    return H;
  }
  // Rows [step, step + nsteps] of a run of time step dt inside the history?
  bool hist_covers(int64_t step, int64_t nsteps, double dt) const {
    const double a = hist_t0 + (double)step * dt, b = hist_t0 + (double)(step + nsteps) * dt;
    return std::min(a, b) >= hist_tmin && std::max(a, b) <= hist_tmax;
  }
  void release_ring() { dfree(d_ring); d_ring = nullptr; ring_rows = 0; ring_slots = 0; }
  void release_base() {
    // the streams belong to the device (shared); only wait for them
    if (sP) (void)hipStreamSynchronize(sP);
    if (sE) (void)hipStreamSynchronize(sE);
    for (int i = 0; i < NSLOT; ++i) {
      if (ev_eph[i]) (void)hipEventDestroy(ev_eph[i]);
      if (ev_done[i]) (void)hipEventDestroy(ev_done[i]);
    }
    for (auto e : {t0P, t1P, t0E, t1E}) if (e) (void)hipEventDestroy(e);
    for (auto e : kev) (void)hipEventDestroy(e);
    for (auto e : ev_cnt) if (e) (void)hipEventDestroy(e);
    dfree(d_flag); dfree(d_nactive); dfree(d_acc);
    if (h_pin) (void)hipHostFree(h_pin);
  }

  SysConst sys() const {
    SysConst S{};
    S.np = np;
    S.mu0 = mu0;
    S.inv_mu0 = 1.0 / mu0;
    S.sqrt_mu0 = std::sqrt(mu0);
    S.inv_sqrt_mu0 = 1.0 / std::sqrt(mu0);
    for (int j = 0; j < np; ++j) {
      S.mu[j] = mu_s[j];
      S.rcrit2[j] = rcrit_s[j] * rcrit_s[j];
    }
    S.rmax2 = opt.r_escape > 0 ? opt.r_escape * opt.r_escape : INFINITY;
    S.kiters = opt.kepler_iters;
    S.ftol = opt.kepler_ftol;
    S.universal = opt.universal_drift ? 1 : 0;
    S.handoff = opt.handoff_substeps > 0 ? 1 : 0;
    return S;
  }

  EphConst eph() const { return make_eph(mu0, np, mu_s.data(), a_s.data()); }
};

namespace {

// Buffers of the close-encounter hand-off for a call of `slots` chunks whose
// ring slots hold `rows` rows: the encounter list (capacity n, empty), the
// list length after each chunk's hand-offs, the planets' velocities per row of
// every slot, the ordering events and the device's encounter stream.
int ensure_handoff(tpm_sim* s, int64_t rows, int64_t slots) {
  DeviceStreams& D = device_streams(s->opt.device);
  if (!D.sH) TPM_HIP(hipStreamCreateWithFlags(&D.sH, hipStreamNonBlocking));
  if (!s->ev_gath[0])
    for (int k = 0; k < NSLOT; ++k) {
      TPM_HIP(hipEventCreateWithFlags(&s->ev_gath[k], hipEventDisableTiming));
      TPM_HIP(hipEventCreateWithFlags(&s->ev_hdone[k], hipEventDisableTiming));
    }
  const size_t n = std::max<int64_t>(s->n, 1);
  if (!s->enc.count) {
    EncList& L = s->enc;
    for (double** p : {&L.x, &L.y, &L.z, &L.vx, &L.vy, &L.vz})
      TPM_HIP(hipMalloc(p, sizeof(double) * n));
    TPM_HIP(hipMalloc(&L.slot, sizeof(int32_t) * n));
    TPM_HIP(hipMalloc(&L.status, sizeof(int32_t) * n));
    TPM_HIP(hipMalloc(&L.step, sizeof(int64_t) * n));
    TPM_HIP(hipMalloc(&L.m, sizeof(int32_t) * n));
    TPM_HIP(hipMalloc(&L.Ml, sizeof(int32_t) * n));
    TPM_HIP(hipMalloc(&L.count, sizeof(int32_t)));
    TPM_HIP(hipMemset(L.count, 0, sizeof(int32_t)));
  }
  if (s->vring_rows < rows || s->vring_slots < slots || s->vring_np != s->np || !s->d_vring ||
      s->snap_slots < slots) {
    TPM_HIP(hipStreamSynchronize(s->sE));
    TPM_HIP(hipStreamSynchronize(s->sP));
    TPM_HIP(hipStreamSynchronize(D.sH));
    dfree(s->d_vring);
    dfree(s->d_snap);
    TPM_HIP(hipMalloc(&s->d_vring, sizeof(double) * slots * rows * 3 * std::max(s->np, 1)));
    TPM_HIP(hipMalloc(&s->d_snap, sizeof(int32_t) * slots));
    s->vring_rows = rows;
    s->vring_slots = slots;
    s->vring_np = s->np;
    s->snap_slots = slots;
  }
  return TPM_OK;
}

int ensure_ring(tpm_sim* s, int64_t rows, int64_t slots = NSLOT) {
  if (s->ring_rows >= rows && s->ring_slots >= slots && s->d_ring) return TPM_OK;
  TPM_HIP(hipStreamSynchronize(s->sE));
  TPM_HIP(hipStreamSynchronize(s->sP));
  s->release_ring();
  size_t bytes = sizeof(double) * (size_t)slots * rows * (3 * s->np + 3);
  TPM_HIP(hipMalloc(&s->d_ring, bytes));
  s->ring_rows = rows;
  s->ring_slots = slots;
  return TPM_OK;
}

// Reorder table columns between caller planet order and internal order.
void permute_table(const tpm_sim* s, const double* src, double* dst, int64_t rows, bool to_caller) {
  const int np = s->np, rl = 3 * np + 3;
  for (int64_t r = 0; r < rows; ++r) {
    const double* a = src + r * rl;
    double* b = dst + r * rl;
    for (int j = 0; j < np; ++j) {
      int c = s->perm[j];
      for (int k = 0; k < 3; ++k) {
        if (to_caller) b[3 * c + k] = a[3 * j + k];
        else b[3 * j + k] = a[3 * c + k];
      }
    }
    for (int k = 0; k < 3; ++k) b[3 * np + k] = a[3 * np + k];
  }
}

// Particle arrays of a simulation from caller-order states and (optionally)
// removal records: results hold every particle, the working set the active
// ones (record reason 0) in caller order.  The device lock is held.
int load_particles(tpm_sim* s, int64_t n, const double* r, const double* v, const int64_t* step,
                   const int32_t* reason, const int32_t* planet) {
  TPM_HIP(hipStreamSynchronize(s->sP));
  s->release_particles();
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  for (auto& w : s->work) {
    TPM_HIP(hipMalloc(&w.x, nn * 8)); TPM_HIP(hipMalloc(&w.y, nn * 8)); TPM_HIP(hipMalloc(&w.z, nn * 8));
    TPM_HIP(hipMalloc(&w.vx, nn * 8)); TPM_HIP(hipMalloc(&w.vy, nn * 8)); TPM_HIP(hipMalloc(&w.vz, nn * 8));
    TPM_HIP(hipMalloc(&w.slot, nn * 4)); TPM_HIP(hipMalloc(&w.status, nn * 4));
  }
  TPM_HIP(hipMalloc(&s->out.r, nn * 24)); TPM_HIP(hipMalloc(&s->out.v, nn * 24));
  TPM_HIP(hipMalloc(&s->out.step, nn * 8)); TPM_HIP(hipMalloc(&s->out.reason, nn * 4));
  TPM_HIP(hipMalloc(&s->out.planet, nn * 4));
  TPM_HIP(hipMalloc(&s->d_scratch, sizeof(int32_t) * compact_scratch_ints((int)nn)));
  const size_t ntiles = (nn + 63) / 64;
  TPM_HIP(hipMalloc(&s->d_qctr, sizeof(unsigned long long)));
  TPM_HIP(hipMalloc(&s->d_progress, sizeof(uint32_t) * ntiles));
  TPM_HIP(hipMalloc(&s->d_qerr, sizeof(int32_t)));
  TPM_HIP(hipMemset(s->d_qctr, 0, sizeof(unsigned long long)));
  TPM_HIP(hipMemset(s->d_progress, 0, sizeof(uint32_t) * ntiles));
  TPM_HIP(hipMemset(s->d_qerr, 0, sizeof(int32_t)));
  TPM_HIP(hipDeviceSynchronize());   // null-stream set-up before work on the non-blocking streams
  // the working set: active particles in caller order, structure of arrays
  std::vector<int32_t> idx;
  idx.reserve(n);
  for (int64_t i = 0; i < n; ++i)
    if (!reason || reason[i] == TPM_ACTIVE) idx.push_back((int32_t)i);
  if (s->opt.sort_by_e && s->central_set) {
    // Expected Newton count grows with eccentricity: bins of 0.1 in the
    // osculating e about mu0 (unbound orbits in the last bin), most eccentric
    // first, caller order within a bin.  The compaction is a stable
    // partition, so the order lasts.
    auto ebin = [&](int32_t i) {
      const double* p = r + 3 * (int64_t)i;
      const double* q = v + 3 * (int64_t)i;
      const double rr = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      const double vv = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
      const double rv = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
      double ev[3];
      for (int k = 0; k < 3; ++k) ev[k] = ((vv - s->mu0 / rr) * p[k] - rv * q[k]) / s->mu0;
      const double e = std::sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
      const double alpha = 2.0 / rr - vv / s->mu0;
      if (!(alpha > 0.0) || !(e < 1.0)) return 10;
      return std::min(9, (int)(e * 10.0));
    };
    std::vector<int> bin(n, 0);
    for (int32_t i : idx) bin[i] = ebin(i);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return bin[a] > bin[b]; });
  }
  const int64_t na = (int64_t)idx.size();
  std::vector<double> col(na);
  Work& w = s->work[0];
  double* dst[6] = {w.x, w.y, w.z, w.vx, w.vy, w.vz};
  for (int c = 0; c < 6; ++c) {
    const double* src = c < 3 ? r : v;
    for (int64_t k = 0; k < na; ++k) col[k] = src[3 * (int64_t)idx[k] + (c % 3)];
    if (na) TPM_HIP(hipMemcpy(dst[c], col.data(), na * 8, hipMemcpyHostToDevice));
  }
  std::vector<int32_t> zero(n, 0), m1(n, -1);
  std::vector<int64_t> m1l(n, -1);
  if (na) {
    TPM_HIP(hipMemcpy(w.slot, idx.data(), na * 4, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(w.status, zero.data(), na * 4, hipMemcpyHostToDevice));
  }
  if (n) {
    TPM_HIP(hipMemcpy(s->out.step, step ? step : m1l.data(), n * 8, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->out.reason, reason ? reason : zero.data(), n * 4, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->out.planet, planet ? planet : m1.data(), n * 4, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->out.r, r, n * 24, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->out.v, v, n * 24, hipMemcpyHostToDevice));
  }
  int32_t na32 = (int32_t)na;
  TPM_HIP(hipMemcpy(s->d_nactive, &na32, 4, hipMemcpyHostToDevice));
  s->cur = 0;
  s->n = n;
  s->n_active = (int)na;
  s->particles_set = true;
  return TPM_OK;
}

int check_eplanet(tpm_sim* s, int rc) {
  if (rc != TPM_OK) return rc;
  int64_t flag = -1;
  TPM_HIP(hipMemcpy(&flag, s->d_flag, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag == -2) return fail(TPM_EPLANET, "a planet orbit became unbound");
  if (flag >= 0)
    return fail(TPM_EPLANET, "two planets came within a mutual Hill radius at step " +
                                 std::to_string(flag));
  return TPM_OK;
}

}  // namespace

extern "C" {

void tpm_default_options(tpm_options* o) {
  if (!o) return;
  o->kepler_iters = 5;
  o->chunk_steps = 0;
  o->resync_chunks = 0;
  o->block_threads = 0;
  o->sub_chunks = 0;
  o->waves_per_simd = 0;
  o->r_escape = 0.0;
  o->kepler_ftol = 0.0;
  o->device = 0;
  o->time_kernels = 0;
  o->universal_drift = 0;
  o->sort_by_e = 0;
  o->handoff_substeps = 0;
}

const char* tpm_last_error(void) { return g_err.c_str(); }

double tpm_hill_radius(double mu0, double mu_p, double a_p) {
  return a_p * std::cbrt(mu_p / (3.0 * mu0));
}

int tpm_create(const tpm_options* opt, tpm_sim** out) {
  if (!out) return fail(TPM_EINVAL, "out is NULL");
  *out = nullptr;
  tpm_options o;
  tpm_default_options(&o);
  if (opt) o = *opt;
  if (o.kepler_iters <= 0) o.kepler_iters = 5;
  if (o.kepler_iters > 64) return fail(TPM_EINVAL, "kepler_iters > 64");
  if (o.chunk_steps < 0 || o.resync_chunks < 0 || o.block_threads < 0 || o.sub_chunks < 0 ||
      o.waves_per_simd < 0)
    return fail(TPM_EINVAL, "negative option");
  if (o.sub_chunks == 0) o.sub_chunks = 64;
  if (o.waves_per_simd > 8) return fail(TPM_EINVAL, "waves_per_simd > 8");
  if (o.chunk_steps == 0) o.chunk_steps = 8192;
  if (o.chunk_steps > (1 << 30)) return fail(TPM_EINVAL, "chunk_steps > 2^30");
  if (o.resync_chunks == 0) o.resync_chunks = 1;
  if (o.block_threads == 0) o.block_threads = 64;
  if (o.block_threads % 64 || o.block_threads > 256)
    return fail(TPM_EINVAL, "block_threads must be 64, 128, 192 or 256");
  if (!(o.kepler_ftol > 0.0)) o.kepler_ftol = 1e-13;
  if (!std::isfinite(o.r_escape)) return fail(TPM_EINVAL, "r_escape not finite");
  if (o.handoff_substeps < 0 || o.handoff_substeps > 4096)
    return fail(TPM_EINVAL, "handoff_substeps must be 0..4096");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(TPM_EDEVICE, "no HIP device");
  if (o.device < 0 || o.device >= ndev) return fail(TPM_EINVAL, "device ordinal out of range");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, o.device) != hipSuccess)
    return fail(TPM_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(TPM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
  TPM_HIP(hipSetDevice(o.device));
  tpm_sim* s = new tpm_sim();
  s->opt = o;
  s->ncu = prop.multiProcessorCount;
  auto bad = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return false;
    fail(TPM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return true;
  };
  {
    DeviceStreams& D = device_streams(o.device);
    if (bad(ensure_device_streams(D), "stream")) {
      delete s;
      return TPM_EDEVICE;
    }
    s->sP = D.sP;
    s->sE = D.sE;
  }
  for (int i = 0; i < NSLOT; ++i)
    if (bad(hipEventCreateWithFlags(&s->ev_eph[i], hipEventDisableTiming), "event") ||
        bad(hipEventCreateWithFlags(&s->ev_done[i], hipEventDisableTiming), "event")) {
      delete s;
      return TPM_EDEVICE;
    }
  if (bad(hipEventCreate(&s->t0P), "event") || bad(hipEventCreate(&s->t1P), "event") ||
      bad(hipEventCreate(&s->t0E), "event") || bad(hipEventCreate(&s->t1E), "event") ||
      bad(hipMalloc(&s->d_flag, sizeof(int64_t)), "alloc") ||
      bad(hipMalloc(&s->d_nactive, sizeof(int32_t)), "alloc") ||
      bad(hipMalloc(&s->d_acc, sizeof(unsigned long long)), "alloc") ||
      bad(hipHostMalloc(&s->h_pin, 256, hipHostMallocDefault), "pinned alloc")) {
    delete s;
    return TPM_EDEVICE;
  }
  for (int i = 0; i < NCNT; ++i)
    if (bad(hipEventCreateWithFlags(&s->ev_cnt[i], hipEventDisableTiming), "event")) {
    delete s;
    return TPM_EDEVICE;
  }
  int64_t m1 = -1;
  if (bad(hipMemcpy(s->d_flag, &m1, sizeof(m1), hipMemcpyHostToDevice), "memcpy")) {
    delete s;
    return TPM_EDEVICE;
  }
  *out = s;
  return TPM_OK;
}

void tpm_destroy(tpm_sim* s) {
  if (!s) return;
  (void)hipSetDevice(s->opt.device);
  delete s;
}

int tpm_set_central(tpm_sim* s, double mu0) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!(std::isfinite(mu0) && mu0 > 0.0)) return fail(TPM_EINVAL, "mu0 must be finite and > 0");
  s->mu0 = mu0;
  s->central_set = true;
  s->planets_set = false;
  return TPM_OK;
}

int tpm_set_planets(tpm_sim* s, int32_t np, const double* mu, const double* r, const double* v,
                    const double* r_crit) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->central_set) return fail(TPM_ESTATE, "tpm_set_central must come first");
  if (np < 0 || np > MAX_NP) return fail(TPM_EINVAL, "np must be in 0..8");
  if (np > 0 && (!mu || !r || !v || !r_crit)) return fail(TPM_EINVAL, "NULL planet array");
  if (np > 0 && !(finite_all(mu, np) && finite_all(r, 3 * np) && finite_all(v, 3 * np) &&
                  finite_all(r_crit, np)))
    return fail(TPM_EINVAL, "planet input not finite");
  std::vector<double> a(np);
  for (int j = 0; j < np; ++j) {
    if (!(mu[j] > 0.0)) return fail(TPM_EINVAL, "planet mu must be > 0");
    if (r_crit[j] < 0.0) return fail(TPM_EINVAL, "r_crit must be >= 0");
    double rr = std::sqrt(r[3 * j] * r[3 * j] + r[3 * j + 1] * r[3 * j + 1] + r[3 * j + 2] * r[3 * j + 2]);
    double vv = v[3 * j] * v[3 * j] + v[3 * j + 1] * v[3 * j + 1] + v[3 * j + 2] * v[3 * j + 2];
    double alpha = 2.0 / rr - vv / (s->mu0 + mu[j]);
    if (!(rr > 0.0) || !(alpha > 0.0)) return fail(TPM_EINVAL, "planet orbit not bound");
    a[j] = 1.0 / alpha;
  }
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sP));
  TPM_HIP(hipStreamSynchronize(s->sE));
  s->release_planets();
  s->release_ring();
  s->np = np;
  s->perm.resize(np);
  std::iota(s->perm.begin(), s->perm.end(), 0);
  std::stable_sort(s->perm.begin(), s->perm.end(), [&](int x, int y) { return a[x] < a[y]; });
  s->mu_s.resize(np);
  s->rcrit_s.resize(np);
  s->a_s.resize(np);
  std::vector<double> rs(3 * np), vs(3 * np);
  for (int j = 0; j < np; ++j) {
    int c = s->perm[j];
    s->mu_s[j] = mu[c];
    s->rcrit_s[j] = r_crit[c];
    s->a_s[j] = a[c];
    for (int k = 0; k < 3; ++k) { rs[3 * j + k] = r[3 * c + k]; vs[3 * j + k] = v[3 * c + k]; }
  }
  size_t b = sizeof(double) * 3 * std::max(np, 1);
  TPM_HIP(hipMalloc(&s->d_rj, b));
  TPM_HIP(hipMalloc(&s->d_vj, b));
  TPM_HIP(hipMalloc(&s->d_tmp, 4 * b));
  if (np > 0) {
    TPM_HIP(hipMemcpy(s->d_tmp, rs.data(), b, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->d_tmp + 3 * np, vs.data(), b, hipMemcpyHostToDevice));
    EphConst E = s->eph();
    TPM_HIP(launch_helio_to_jacobi(E, s->d_tmp, s->d_rj, s->sE));
    TPM_HIP(launch_helio_to_jacobi(E, s->d_tmp + 3 * np, s->d_vj, s->sE));
    TPM_HIP(hipStreamSynchronize(s->sE));
  }
  int64_t m1 = -1;
  TPM_HIP(hipMemcpy(s->d_flag, &m1, sizeof(m1), hipMemcpyHostToDevice));
  s->step = 0;
  s->planets_set = true;
  s->rrem_set = false;
  return TPM_OK;
}

int tpm_set_removal_radii(tpm_sim* s, const double* r_rem) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "tpm_set_planets must come first");
  if (s->np > 0 && !r_rem) return fail(TPM_EINVAL, "r_rem is NULL");
  std::vector<double> r(s->np);
  for (int j = 0; j < s->np; ++j) {
    const double v = r_rem[s->perm[j]];
    if (!(std::isfinite(v) && v > 0.0)) return fail(TPM_EINVAL, "removal radius must be > 0");
    r[j] = v;
  }
  s->rrem_s = r;
  s->rrem_set = true;
  return TPM_OK;
}

int tpm_set_particles(tpm_sim* s, int64_t n, const double* r, const double* v) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(TPM_EINVAL, "n out of range");
  if (n > 0 && (!r || !v)) return fail(TPM_EINVAL, "NULL particle array");
  if (n > 0 && !(finite_all(r, 3 * n) && finite_all(v, 3 * n)))
    return fail(TPM_EINVAL, "particle input not finite");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  return load_particles(s, n, r, v, nullptr, nullptr, nullptr);
}

int tpm_set_planet_table(tpm_sim* s, const double* table, int64_t nrows) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "tpm_set_planets must come first");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sP));
  TPM_HIP(hipStreamSynchronize(s->sE));
  dfree(s->d_table);
  s->d_table = nullptr;
  s->table_rows = 0;
  if (nrows <= 0) return TPM_OK;
  s->release_history();
  if (!table) return fail(TPM_EINVAL, "table is NULL");
  const int rl = 3 * s->np + 3;
  if (!finite_all(table, nrows * rl)) return fail(TPM_EINVAL, "table not finite");
  std::vector<double> t(nrows * rl);
  permute_table(s, table, t.data(), nrows, false);
  TPM_HIP(hipMalloc(&s->d_table, sizeof(double) * t.size()));
  TPM_HIP(hipMemcpy(s->d_table, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
  s->table_rows = nrows;
  return TPM_OK;
}

int tpm_set_planet_history(tpm_sim* s, int64_t nrec, const double* t, const double* r,
                           const double* v, double t0) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "tpm_set_planets must come first");
  const int np = s->np;
  if (nrec > 0) {
    if (!t || (np > 0 && (!r || !v))) return fail(TPM_EINVAL, "NULL history array");
    if (nrec > (int64_t(1) << 40) / std::max(1, 6 * np + 1))
      return fail(TPM_EINVAL, "history too long");
    if (!finite_all(t, nrec) || !finite_all(r, 3 * np * nrec) || !finite_all(v, 3 * np * nrec) ||
        !std::isfinite(t0))
      return fail(TPM_EINVAL, "history not finite");
    for (int64_t k = 1; k < nrec; ++k)
      if (!(t[k] > t[k - 1])) return fail(TPM_EINVAL, "history times must increase");
  }
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sP));
  TPM_HIP(hipStreamSynchronize(s->sE));
  s->release_history();
  if (nrec <= 0) return TPM_OK;
  dfree(s->d_table);
  s->table_rows = 0;
  // records in the integration order of the planets
  std::vector<double> h((size_t)nrec * (1 + 6 * np));
  std::memcpy(h.data(), t, sizeof(double) * nrec);
  double* hr = h.data() + nrec;
  double* hv = hr + (size_t)nrec * 3 * np;
  for (int64_t k = 0; k < nrec; ++k)
    for (int j = 0; j < np; ++j)
      for (int c = 0; c < 3; ++c) {
        hr[(k * np + j) * 3 + c] = r[(k * np + s->perm[j]) * 3 + c];
        hv[(k * np + j) * 3 + c] = v[(k * np + s->perm[j]) * 3 + c];
      }
  TPM_HIP(hipMalloc(&s->d_hist, sizeof(double) * h.size()));
  TPM_HIP(hipMemcpy(s->d_hist, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  s->hist_nrec = nrec;
  s->hist_t0 = t0;
  s->hist_tmin = t[0];
  s->hist_tmax = t[nrec - 1];
  return TPM_OK;
}

int tpm_integrate(tpm_sim* s, int64_t nsteps, double dt) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set || !s->particles_set)
    return fail(TPM_ESTATE, "set central mass, planets and particles first");
  if (nsteps < 0) return fail(TPM_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt) || dt == 0.0) return fail(TPM_EINVAL, "dt must be finite and non-zero");
  if (s->d_table && s->step + nsteps > s->table_rows - 1)
    return fail(TPM_EINVAL, "supplied planet table too short");
  if (s->d_hist && !s->hist_covers(s->step, nsteps, dt))
    return fail(TPM_EINVAL, "the run's row times leave the planet history");
  if (s->opt.handoff_substeps > 0 && !s->d_table && !s->d_hist) {
    const int64_t K = s->opt.chunk_steps;
    const int64_t per_slot = (K + 1) * (3 * s->np + 3 + 3 * std::max(s->np, 1)) * 8;
    const int64_t max_slots = std::max<int64_t>(2, handoff_ring_bytes() / per_slot);
    const int64_t seg = std::min<int64_t>(K, FIRST_CHUNK_STEPS) + (max_slots - 1) * K;
    if (nsteps > seg) {
      tpm_stats agg = s->stats;
      agg.chunks = agg.compactions = agg.handoffs = agg.active_particle_steps = 0;
      agg.particle_kernel_ms = agg.particle_ms = agg.ephemeris_ms = agg.wall_ms = 0.0;
      int ret = TPM_OK;
      for (int64_t done = 0; done < nsteps;) {
        const int64_t piece = std::min(seg, nsteps - done);
        const int rc = tpm_integrate(s, piece, dt);
        if (rc != TPM_OK && rc != TPM_EPLANET) return rc;
        if (rc == TPM_EPLANET) ret = rc;
        agg.chunks += s->stats.chunks;
        agg.compactions += s->stats.compactions;
        agg.handoffs += s->stats.handoffs;
        agg.active_particle_steps += s->stats.active_particle_steps;
        agg.particle_kernel_ms += s->stats.particle_kernel_ms;
        agg.particle_ms += s->stats.particle_ms;
        agg.ephemeris_ms += s->stats.ephemeris_ms;
        agg.wall_ms += s->stats.wall_ms;
        done += piece;
      }
      s->stats = agg;
      return ret;
    }
  }
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  auto w0 = std::chrono::steady_clock::now();
  const int K = s->opt.chunk_steps;
  const int R = s->opt.resync_chunks;
  const int rl = 3 * s->np + 3;
  // The particles wait for the whole first chunk of the planet map before
  // they start, so when the map runs on the fly the first chunk is short;
  // chunk c covers steps [begin(c), begin(c + 1)) of this call.
  const int K0 = (s->d_table || s->d_hist) ? K : std::min(K, FIRST_CHUNK_STEPS);
  auto& D = s->diag;
  if (D.on && D.nres > 0 && s->d_table)
    return fail(TPM_ESTATE, "resonant angles need planet velocities, which a supplied planet "
                            "table does not carry");
  const bool ho = s->opt.handoff_substeps > 0;
  if (ho) {
    if (!s->rrem_set) return fail(TPM_ESTATE, "the hand-off needs removal radii (tpm_set_removal_radii)");
    if (s->d_table || s->d_hist)
      return fail(TPM_ESTATE, "the hand-off needs the on-device planet map (its planet velocities)");
    if (D.on) return fail(TPM_ESTATE, "diagnostics and the hand-off do not run together");
  }
  // Chunk c covers steps [cb[c], cb[c + 1]) of this call: the first K0 steps
  // long, the others K, each also ending at every sample boundary (global
  // steps that are multiples of the diagnostics interval).
  std::vector<int64_t> cb{0};
  while (cb.back() < nsteps) {
    const int64_t b = cb.back();
    int64_t e = std::min(nsteps, b + (cb.size() == 1 ? K0 : K));
    if (D.on) e = std::min(e, ((s->step + b) / D.every + 1) * D.every - s->step);
    cb.push_back(e);
  }
  auto begin = [&](int64_t c) -> int64_t { return cb[c]; };
  auto length = [&](int64_t c) -> int { return (int)(cb[c + 1] - cb[c]); };
  const int64_t nchunks = (int64_t)cb.size() - 1;
  // With the hand-off the ring keeps every chunk of the call (slot c for chunk
  // c), so that the encounter stream may lag behind the particle stream.
  const int64_t ring_slots = ho ? std::max<int64_t>(nchunks, 1) : NSLOT;
  auto row_slot = [&](int64_t c) -> int64_t { return ho ? c : c % NSLOT; };
  if (!s->d_table) {
    int rc = ensure_ring(s, (int64_t)K + 1, ring_slots);
    if (rc) return rc;
  }
  hipStream_t sH = nullptr;
  double rrem2[MAX_NP] = {};
  if (ho) {
    int rc = ensure_handoff(s, s->ring_rows, ring_slots);
    if (rc) return rc;
    sH = device_streams(s->opt.device).sH;
    for (int j = 0; j < s->np; ++j) rrem2[j] = s->rrem_s[j] * s->rrem_s[j];
  }
  const SysConst S = s->sys();
  const EphConst E = s->eph();
  const int64_t step_begin = s->step;
  const bool timed = s->opt.time_kernels != 0;
  if (timed) {
    while ((int64_t)s->kev.size() < 2 * nchunks) {
      hipEvent_t e;
      TPM_HIP(hipEventCreate(&e));
      s->kev.push_back(e);
    }
  }
  s->stats.chunks = 0;
  s->stats.compactions = 0;
  TPM_HIP(hipEventRecord(s->t0P, s->sP));
  TPM_HIP(hipEventRecord(s->t0E, s->sE));
  // The planet map is enqueued up to NSLOT-1 chunks ahead of the particles so
  // that it keeps running while the host waits on anything else.
  int64_t eph_next = 0;
  auto enqueue_eph = [&](int64_t upto) -> int {
    for (; eph_next <= upto && eph_next < nchunks; ++eph_next) {
      const int64_t c = eph_next;
      const int ks = length(c);
      const int slot = (int)(c % NSLOT);
      double* srow = s->d_ring + (size_t)row_slot(c) * s->ring_rows * rl;
      TPM_HIP(hipStreamWaitEvent(s->sE, s->ev_done[slot], 0));
      double* vs = s->d_vside ? s->d_vside + (size_t)slot * 6 * s->np : nullptr;
      // with the hand-off, the planets' velocities at every row too (for the
      // encounter integrator's interpolation; the slot is this chunk's alone)
      double* vr = ho ? s->d_vring + (size_t)c * s->vring_rows * 3 * s->np : nullptr;
      if (s->d_hist)
        TPM_HIP(launch_history_rows(s->hist(), srow, ks + 1, s->step + begin(c), dt, vs, s->sE));
      else
        TPM_HIP(launch_ephemeris_chunk(E, s->d_rj, s->d_vj, srow, ks, dt, s->step + begin(c),
                                       s->d_flag, s->sE, vs, vr));
      TPM_HIP(hipEventRecord(s->ev_eph[slot], s->sE));
    }
    return TPM_OK;
  };
  // Newest active count whose readback has completed (never blocks); the
  // count is only an upper bound for the grid, the kernels read the exact
  // value on the device.
  auto poll_counts = [&]() -> int {
    while (s->cnt_seen < s->cnt_issued) {
      hipEvent_t e = s->ev_cnt[s->cnt_seen % NCNT];
      hipError_t q = hipEventQuery(e);
      if (q == hipErrorNotReady) break;
      TPM_HIP(q);
      s->n_active = std::min(s->n_active, (int)s->h_pin[s->cnt_seen % NCNT]);
      s->cnt_seen++;
    }
    return TPM_OK;
  };
  // Snapshots copied to the pinned ring, in order, waiting for their callbacks.
  std::deque<std::pair<int, int64_t>> pend;     // (ring buffer, step)
  int64_t snaps = 0;
  auto fire = [&](bool block, size_t upto) -> int {   // hand out at most `upto`, in order
    for (; !pend.empty() && upto > 0; --upto) {
      const int k = pend.front().first;
      if (block) {
        TPM_HIP(hipEventSynchronize(D.ev_snap[k]));
      } else {
        hipError_t q = hipEventQuery(D.ev_snap[k]);
        if (q == hipErrorNotReady) break;
        TPM_HIP(q);
      }
      const int64_t n = s->n;
      const char* h = D.h_snap[k];
      D.snap(D.user, pend.front().second, n, (const double*)h, (const double*)(h + 24 * n),
             (const int64_t*)(h + 96 * n), (const int32_t*)(h + 104 * n),
             (const double*)(h + 48 * n));
      pend.pop_front();
    }
    return TPM_OK;
  };
  // Sample (and snapshot) the state at global step `gstep`, whose table row is
  // `row` and planet velocities (internal order) `vel`.
  auto sample = [&](int64_t gstep, const double* row, const double* vel, int n_upper) -> int {
    DiagArgs A{};
    A.emax = D.emax; A.estep = D.estep; A.flags = D.flags; A.lo = D.lo; A.hi = D.hi;
    A.nres = D.nres;
    for (int k = 0; k < 2; ++k) { A.p[k] = D.p[k]; A.q[k] = D.q[k]; }
    A.ref = D.ref;
    A.mu0 = s->mu0;
    A.mu_ref = D.ref >= 0 ? s->mu0 + s->mu_s[D.ref] : s->mu0;
    A.vref = (vel && D.ref >= 0) ? vel + 3 * D.ref : nullptr;
    const int64_t n = s->n;
    if (D.snap) {
      A.snap_r = (double*)D.d_snap;
      A.snap_v = (double*)(D.d_snap + 24 * n);
      A.snap_el = (double*)(D.d_snap + 48 * n);
      A.snap_step = (int64_t*)(D.d_snap + 96 * n);
      A.snap_reason = (int32_t*)(D.d_snap + 104 * n);
      TPM_HIP(launch_snapshot_base(s->out, (int)n, s->mu0, A, s->sP));
    }
    TPM_HIP(launch_sample(S, s->work[s->cur], s->d_nactive, n_upper, row, gstep, A, s->sP));
    if (D.snap) {
      const int k = (int)(snaps % 2);
      if (pend.size() == 2) {                  // ring full: hand out the oldest first
        int rc = fire(true, 1);
        if (rc) return rc;
      }
      TPM_HIP(hipMemcpyAsync(D.h_snap[k], D.d_snap, (size_t)108 * n, hipMemcpyDeviceToHost,
                             s->sP));
      TPM_HIP(hipEventRecord(D.ev_snap[k], s->sP));
      pend.emplace_back(k, gstep);
      snaps++;
    }
    D.last_step = gstep;
    return TPM_OK;
  };
  int n_grid = s->n_active;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int ks = length(c);
    const int slot = (int)(c % NSLOT);
    const int64_t step0 = s->step + begin(c);
    const double* rows;
    if (s->d_table) {
      rows = s->d_table + (size_t)step0 * rl;
    } else {
      int rc = enqueue_eph(c + NSLOT - 1);
      if (rc) return rc;
      TPM_HIP(hipStreamWaitEvent(s->sP, s->ev_eph[slot], 0));
      rows = s->d_ring + (size_t)row_slot(c) * s->ring_rows * rl;
    }
    {
      int rc = poll_counts();
      if (rc) return rc;
      n_grid = std::min(n_grid, s->n_active);
    }
    const double* vel = s->d_vside ? s->d_vside + (size_t)slot * 6 * s->np : nullptr;
    if (c == 0 && D.on && step0 % D.every == 0 && step0 != D.last_step) {
      int rc = sample(step0, rows, vel, n_grid);
      if (rc) return rc;
    }
    if (n_grid > 0) {
      Work& w = s->work[s->cur];
      if (timed) TPM_HIP(hipEventRecord(s->kev[2 * s->stats.chunks], s->sP));
      QueueLaunch QL;
      QL.ctr = s->d_qctr;
      QL.base = s->q_base;
      QL.progress = s->d_progress;
      QL.epoch = s->q_epoch;
      // items keep the length of a full chunk's (K / sub_chunks steps): a short
      // chunk gets fewer items, not shorter ones
      const int item = std::max(1, K / std::max(1, s->opt.sub_chunks));
      QL.nsub = std::max(1, std::min(s->opt.sub_chunks, (ks + item - 1) / item));
      const int ntiles = (n_grid + 63) / 64;
      const int wps = s->opt.waves_per_simd > 0 ? s->opt.waves_per_simd
                                                 : auto_waves_per_simd(ntiles, s->ncu);
      s->last_wps = wps;
      QL.workers = std::max(1, std::min(ntiles * QL.nsub, 4 * s->ncu * wps));
      QL.deep = wps == 1 && !ho;
      QL.workers = std::min(QL.workers, ntiles);
      QL.block = s->opt.block_threads;
      QL.error = s->d_qerr;
      TPM_HIP(launch_particle_chunk(S, w, s->d_nactive, n_grid, s->out, rows, ks, dt, step0, QL,
                                    s->sP));
      // every wavefront takes exactly one failing item at the end
      const int wpb = QL.block / 64;
      const unsigned long long waves = (unsigned long long)((QL.workers + wpb - 1) / wpb) * wpb;
      s->q_base += (unsigned long long)ntiles * QL.nsub + waves;
      s->q_epoch += (uint32_t)QL.nsub;
      if (timed) TPM_HIP(hipEventRecord(s->kev[2 * s->stats.chunks + 1], s->sP));
      s->stats.chunks++;
    }
    if (D.on && (step0 + ks) % D.every == 0) {
      int rc = sample(step0 + ks, rows + (size_t)ks * rl, vel ? vel + 3 * s->np : nullptr, n_grid);
      if (rc) return rc;
      rc = fire(false, SIZE_MAX);
      if (rc) return rc;
    }
    if (ho) {
      // particles handed off in this chunk join the encounter list, which the
      // encounter stream advances towards the chunk's end while the particle
      // stream goes on: a budget of micro-steps per entry (the chunk's length)
      // keeps each launch about as long as a particle launch, and an entry
      // left behind is resumed by the next launch; the call's last launch
      // takes every entry to the end
      TPM_HIP(launch_handoff_gather(s->work[s->cur], s->d_nactive, n_grid, s->enc, step0,
                                    s->d_snap + c, s->sP));
      TPM_HIP(hipEventRecord(s->ev_gath[slot], s->sP));
      TPM_HIP(hipStreamWaitEvent(sH, s->ev_gath[slot], 0));
      EncRing ER;
      ER.rows = s->d_ring;
      ER.vrows = s->d_vring;
      ER.ring_rows = s->ring_rows;
      ER.vring_rows = s->vring_rows;
      ER.k0 = K0;
      ER.k = K;
      ER.nsteps = nsteps;
      ER.step0 = s->step;
      const int64_t budget = (c == nchunks - 1) ? 0 : (int64_t)K;
      TPM_HIP(launch_encounter_run(S, rrem2, s->enc, s->d_snap + c, (int)s->n, ER, begin(c + 1),
                                   budget, dt, s->opt.handoff_substeps, s->out, sH));
      TPM_HIP(hipEventRecord(s->ev_hdone[slot], sH));
    }
    TPM_HIP(hipEventRecord(s->ev_done[slot], s->sP));
    const bool last = (c == nchunks - 1);
    if (n_grid > 0 && (((c + 1) % R == 0) || last)) {
      Work& src = s->work[s->cur];
      Work& dst = s->work[1 - s->cur];
      TPM_HIP(launch_compact(src, dst, s->d_nactive, n_grid, s->d_scratch, s->sP));
      s->cur = 1 - s->cur;
      s->stats.compactions++;
      if (s->cnt_issued - s->cnt_seen >= NCNT) {       // ring full: wait for the oldest
        TPM_HIP(hipEventSynchronize(s->ev_cnt[s->cnt_seen % NCNT]));
        int rc = poll_counts();
        if (rc) return rc;
      }
      const int k = (int)(s->cnt_issued % NCNT);
      TPM_HIP(hipMemcpyAsync(s->h_pin + k, s->d_nactive, 4, hipMemcpyDeviceToHost, s->sP));
      TPM_HIP(hipEventRecord(s->ev_cnt[k], s->sP));
      s->cnt_issued++;
    }
  }
  if (ho && nchunks > 0) {
    // the encounter list's survivors rejoin the working set (every entry is
    // now at the run's last step); the list ends the call empty
    TPM_HIP(hipStreamWaitEvent(s->sP, s->ev_hdone[(nchunks - 1) % NSLOT], 0));
    TPM_HIP(hipMemcpyAsync(s->h_pin + 18, s->enc.count, sizeof(int32_t), hipMemcpyDeviceToHost,
                           s->sP));
    TPM_HIP(launch_handoff_merge(s->enc, (int)s->n, s->work[s->cur], s->d_nactive, s->sP));
    TPM_HIP(hipMemcpyAsync(s->h_pin + 19, s->d_nactive, sizeof(int32_t), hipMemcpyDeviceToHost,
                           s->sP));
  }
  TPM_HIP(hipEventRecord(s->t1P, s->sP));
  TPM_HIP(hipEventRecord(s->t1E, s->sE));
  TPM_HIP(hipStreamSynchronize(s->sE));
  TPM_HIP(hipStreamSynchronize(s->sP));
  {
    int rc = poll_counts();
    if (rc) return rc;
    rc = fire(true, SIZE_MAX);
    if (rc) return rc;
  }
  s->stats.handoffs = 0;
  if (ho && nchunks > 0) {
    s->stats.handoffs = s->h_pin[18];
    s->n_active = s->h_pin[19];
  }
  {
    int32_t qerr = 0;
    TPM_HIP(hipMemcpy(&qerr, s->d_qerr, sizeof(qerr), hipMemcpyDeviceToHost));
    if (qerr) return fail(TPM_EDEVICE, "particle work queue: a wait exceeded its limit");
  }
  s->step += nsteps;
  s->hist_dt = dt;
  float msP = 0.f, msE = 0.f;
  TPM_HIP(hipEventElapsedTime(&msP, s->t0P, s->t1P));
  TPM_HIP(hipEventElapsedTime(&msE, s->t0E, s->t1E));
  // active particle-steps of this call
  TPM_HIP(hipMemsetAsync(s->d_acc, 0, sizeof(unsigned long long), s->sP));
  TPM_HIP(launch_active_steps(s->out.step, (int)s->n, step_begin, s->step, s->d_acc, s->sP));
  unsigned long long acc = 0;
  TPM_HIP(hipMemcpyAsync(s->h_pin + 16, s->d_acc, sizeof(acc), hipMemcpyDeviceToHost, s->sP));
  TPM_HIP(hipStreamSynchronize(s->sP));
  std::memcpy(&acc, s->h_pin + 16, sizeof(acc));
  auto w1 = std::chrono::steady_clock::now();
  double kms = 0.0;
  if (timed)
    for (int64_t c = 0; c < s->stats.chunks; ++c) {
      float m = 0.f;
      TPM_HIP(hipEventElapsedTime(&m, s->kev[2 * c], s->kev[2 * c + 1]));
      kms += m;
    }
  s->stats.particle_kernel_ms = kms;
  s->stats.particle_ms = msP;
  s->stats.ephemeris_ms = msE;
  s->stats.wall_ms = std::chrono::duration<double, std::milli>(w1 - w0).count();
  s->stats.active_particle_steps = (int64_t)acc;
  return check_eplanet(s, TPM_OK);
}

int tpm_get_particles(tpm_sim* s, double* r, double* v, int64_t* deact_step, int32_t* reason,
                      int32_t* planet) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->particles_set) return fail(TPM_ESTATE, "no particles");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  const int64_t n = s->n;
  if (n == 0) return TPM_OK;
  TPM_HIP(launch_finalize(s->work[s->cur], s->d_nactive, s->n_active, s->out, s->sP));
  TPM_HIP(hipStreamSynchronize(s->sP));
  if (r) TPM_HIP(hipMemcpy(r, s->out.r, n * 24, hipMemcpyDeviceToHost));
  if (v) TPM_HIP(hipMemcpy(v, s->out.v, n * 24, hipMemcpyDeviceToHost));
  if (deact_step) TPM_HIP(hipMemcpy(deact_step, s->out.step, n * 8, hipMemcpyDeviceToHost));
  if (reason) TPM_HIP(hipMemcpy(reason, s->out.reason, n * 4, hipMemcpyDeviceToHost));
  if (planet) {
    TPM_HIP(hipMemcpy(planet, s->out.planet, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i)
      if (planet[i] >= 0) planet[i] = s->perm[planet[i]];
  }
  return TPM_OK;
}

int tpm_set_diagnostics(tpm_sim* s, const tpm_diag_options* o) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->particles_set || !s->planets_set)
    return fail(TPM_ESTATE, "set planets and particles before the diagnostics");
  if (o && o->every < 0) return fail(TPM_EINVAL, "every < 0");
  int ref = -1;
  if (o && o->every > 0) {
    if (o->nres < 0 || o->nres > 2) return fail(TPM_EINVAL, "nres must be 0, 1 or 2");
    for (int k = 0; k < o->nres; ++k)
      if (o->p[k] <= 0 || o->q[k] <= 0 || o->p[k] > 1000 || o->q[k] > 1000)
        return fail(TPM_EINVAL, "resonance p:q needs 0 < p, q <= 1000");
    if (o->nres > 0) {
      if (o->ref_planet < 0 || o->ref_planet >= s->np)
        return fail(TPM_EINVAL, "reference planet out of range");
      for (int j = 0; j < s->np; ++j)
        if (s->perm[j] == o->ref_planet) ref = j;
    }
  }
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  s->release_diag();
  if (!o || o->every == 0) return TPM_OK;
  auto& D = s->diag;
  const int64_t n = std::max<int64_t>(s->n, 1);
  const int nr = std::max(o->nres, 1);
  TPM_HIP(hipMalloc(&D.emax, n * 8));
  TPM_HIP(hipMalloc(&D.estep, n * 8));
  TPM_HIP(hipMalloc(&D.flags, n * nr * 4));
  TPM_HIP(hipMalloc(&D.lo, n * nr * 8));
  TPM_HIP(hipMalloc(&D.hi, n * nr * 8));
  if (o->nres > 0) TPM_HIP(hipMalloc(&s->d_vside, sizeof(double) * NSLOT * 6 * s->np));
  if (o->snapshot) {
    TPM_HIP(hipMalloc(&D.d_snap, 108 * n));
    for (int k = 0; k < 2; ++k) {
      TPM_HIP(hipHostMalloc(&D.h_snap[k], 108 * n, hipHostMallocDefault));
      TPM_HIP(hipEventCreateWithFlags(&D.ev_snap[k], hipEventDisableTiming));
    }
  }
  D.every = o->every;
  D.nres = o->nres;
  D.ref = ref;
  for (int k = 0; k < 2; ++k) {
    D.p[k] = k < o->nres ? o->p[k] : 0;
    D.q[k] = k < o->nres ? o->q[k] : 0;
  }
  D.snap = o->snapshot;
  D.user = o->user;
  DiagArgs A{};
  A.emax = D.emax; A.estep = D.estep; A.flags = D.flags; A.lo = D.lo; A.hi = D.hi;
  A.nres = D.nres;
  TPM_HIP(launch_diag_reset((int)s->n, A, s->sP));
  TPM_HIP(hipStreamSynchronize(s->sP));
  D.on = true;
  return TPM_OK;
}

int tpm_get_diagnostics(tpm_sim* s, double* emax, int64_t* emax_step, int32_t* flags,
                        double* phi_lo, double* phi_hi) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->diag.on) return fail(TPM_ESTATE, "diagnostics are off");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sP));
  const int64_t n = s->n, m = n * s->diag.nres;
  if (n == 0) return TPM_OK;
  if (emax) TPM_HIP(hipMemcpy(emax, s->diag.emax, n * 8, hipMemcpyDeviceToHost));
  if (emax_step) TPM_HIP(hipMemcpy(emax_step, s->diag.estep, n * 8, hipMemcpyDeviceToHost));
  if (m && flags) TPM_HIP(hipMemcpy(flags, s->diag.flags, m * 4, hipMemcpyDeviceToHost));
  if (m && phi_lo) TPM_HIP(hipMemcpy(phi_lo, s->diag.lo, m * 8, hipMemcpyDeviceToHost));
  if (m && phi_hi) TPM_HIP(hipMemcpy(phi_hi, s->diag.hi, m * 8, hipMemcpyDeviceToHost));
  return TPM_OK;
}

int tpm_get_planets(tpm_sim* s, double* r, double* v) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "no planets");
  const int np = s->np;
  if (np == 0) return TPM_OK;
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sE));
  std::vector<double> h(6 * np);
  if (s->d_hist) {
    // the history's state at the current step (time t0 + step dt of the last
    // integrate's dt)
    if (!s->hist_covers(s->step, 0, s->hist_dt))
      return fail(TPM_EINVAL, "the current step's time lies outside the planet history");
    double* row = s->d_tmp;                     // 3 np + 3
    double* vel = s->d_tmp + 3 * np + 3;        // [2][np][3]
    TPM_HIP(launch_history_rows(s->hist(), row, 1, s->step, s->hist_dt, vel, s->sE));
    TPM_HIP(hipMemcpyAsync(h.data(), row, sizeof(double) * 3 * np, hipMemcpyDeviceToHost, s->sE));
    TPM_HIP(hipMemcpyAsync(h.data() + 3 * np, vel, sizeof(double) * 3 * np, hipMemcpyDeviceToHost,
                           s->sE));
  } else {
    TPM_HIP(launch_jacobi_to_helio(s->eph(), s->d_rj, s->d_vj, s->d_tmp, s->d_tmp + 3 * np, s->sE));
    TPM_HIP(hipMemcpyAsync(h.data(), s->d_tmp, sizeof(double) * 6 * np, hipMemcpyDeviceToHost,
                           s->sE));
  }
  TPM_HIP(hipStreamSynchronize(s->sE));
  for (int j = 0; j < np; ++j) {
    int c = s->perm[j];
    for (int k = 0; k < 3; ++k) {
      if (r) r[3 * c + k] = h[3 * j + k];
      if (v) v[3 * c + k] = h[3 * np + 3 * j + k];
    }
  }
  return TPM_OK;
}

}  // extern "C"

namespace {

// Layout of the state blob of tpm_get_state / tpm_set_state: this header, then
// r[n][3], v[n][3] (f64), step[n] (i64), reason[n], planet[n] (i32, planet in
// the integration's sorted order), all native-endian.
struct StateHeader {
  char magic[8];
  int32_t version;
  int32_t np;
  int64_t n;
  int64_t step;
  int64_t flag;                  // first planet event so far (-1 none)
  double mu0;
  int32_t perm[MAX_NP];          // sorted planet index -> caller index
  double mu[MAX_NP], rcrit[MAX_NP], a[MAX_NP];   // sorted order
  double rj[3 * MAX_NP], vj[3 * MAX_NP];         // Jacobi planet state
};
constexpr char STATE_MAGIC[8] = {'t', 'p', 'm', 's', 't', 'a', 't', 'e'};
constexpr int32_t STATE_VERSION = 1;

int64_t state_bytes(int64_t n) { return (int64_t)sizeof(StateHeader) + 64 * n; }

}  // namespace

extern "C" {

int tpm_get_state(tpm_sim* s, void* buf, int64_t* size) {
  if (!s || !size) return fail(TPM_EINVAL, "NULL argument");
  if (!s->planets_set || !s->particles_set)
    return fail(TPM_ESTATE, "set central mass, planets and particles first");
  const int64_t n = s->n, need = state_bytes(n);
  if (!buf) {
    *size = need;
    return TPM_OK;
  }
  if (*size < need) return fail(TPM_EINVAL, "state buffer too small");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sE));
  TPM_HIP(hipStreamSynchronize(s->sP));
  StateHeader h{};
  std::memcpy(h.magic, STATE_MAGIC, 8);
  h.version = STATE_VERSION;
  h.np = s->np;
  h.n = n;
  h.step = s->step;
  h.mu0 = s->mu0;
  TPM_HIP(hipMemcpy(&h.flag, s->d_flag, sizeof(int64_t), hipMemcpyDeviceToHost));
  for (int j = 0; j < s->np; ++j) {
    h.perm[j] = s->perm[j];
    h.mu[j] = s->mu_s[j];
    h.rcrit[j] = s->rcrit_s[j];
    h.a[j] = s->a_s[j];
  }
  if (s->np > 0) {
    TPM_HIP(hipMemcpy(h.rj, s->d_rj, sizeof(double) * 3 * s->np, hipMemcpyDeviceToHost));
    TPM_HIP(hipMemcpy(h.vj, s->d_vj, sizeof(double) * 3 * s->np, hipMemcpyDeviceToHost));
  }
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  if (n > 0) {
    TPM_HIP(launch_finalize(s->work[s->cur], s->d_nactive, s->n_active, s->out, s->sP));
    TPM_HIP(hipStreamSynchronize(s->sP));
    TPM_HIP(hipMemcpy(p, s->out.r, n * 24, hipMemcpyDeviceToHost)); p += n * 24;
    TPM_HIP(hipMemcpy(p, s->out.v, n * 24, hipMemcpyDeviceToHost)); p += n * 24;
    TPM_HIP(hipMemcpy(p, s->out.step, n * 8, hipMemcpyDeviceToHost)); p += n * 8;
    TPM_HIP(hipMemcpy(p, s->out.reason, n * 4, hipMemcpyDeviceToHost)); p += n * 4;
    TPM_HIP(hipMemcpy(p, s->out.planet, n * 4, hipMemcpyDeviceToHost));
  }
  *size = need;
  return TPM_OK;
}

int tpm_set_state(tpm_sim* s, const void* buf, int64_t size) {
  if (!s || !buf) return fail(TPM_EINVAL, "NULL argument");
  if (size < (int64_t)sizeof(StateHeader)) return fail(TPM_EINVAL, "state blob too short");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, STATE_MAGIC, 8) != 0 || h.version != STATE_VERSION)
    return fail(TPM_EINVAL, "not a state blob of this library version");
  if (h.np < 0 || h.np > MAX_NP || h.n < 0 || h.n >= (int64_t(1) << 31) ||
      size != state_bytes(h.n))
    return fail(TPM_EINVAL, "state blob sizes inconsistent");
  const int np = h.np;
  const int64_t n = h.n;
  if (!(std::isfinite(h.mu0) && h.mu0 > 0.0)) return fail(TPM_EINVAL, "state: bad mu0");
  {
    std::vector<int> seen(np, 0);
    for (int j = 0; j < np; ++j) {
      if (h.perm[j] < 0 || h.perm[j] >= np || seen[h.perm[j]]++)
        return fail(TPM_EINVAL, "state: bad planet order");
      if (!(h.mu[j] > 0.0 && std::isfinite(h.mu[j]) && h.rcrit[j] >= 0.0 &&
            std::isfinite(h.rcrit[j]) && h.a[j] > 0.0 && std::isfinite(h.a[j])))
        return fail(TPM_EINVAL, "state: bad planet constants");
    }
    if (!finite_all(h.rj, 3 * np) || !finite_all(h.vj, 3 * np))
      return fail(TPM_EINVAL, "state: planet state not finite");
  }
  const char* p = static_cast<const char*>(buf) + sizeof(StateHeader);
  std::vector<double> r(3 * n), v(3 * n);
  std::vector<int64_t> step(n);
  std::vector<int32_t> reason(n), planet(n);
  if (n > 0) {
    std::memcpy(r.data(), p, n * 24); p += n * 24;
    std::memcpy(v.data(), p, n * 24); p += n * 24;
    std::memcpy(step.data(), p, n * 8); p += n * 8;
    std::memcpy(reason.data(), p, n * 4); p += n * 4;
    std::memcpy(planet.data(), p, n * 4);
  }
  if (!finite_all(r.data(), 3 * n) || !finite_all(v.data(), 3 * n))
    return fail(TPM_EINVAL, "state: particle state not finite");
  for (int64_t i = 0; i < n; ++i)
    if (reason[i] < TPM_ACTIVE || reason[i] > TPM_KEPLER || planet[i] < -1 || planet[i] >= np)
      return fail(TPM_EINVAL, "state: bad removal record");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  TPM_HIP(hipStreamSynchronize(s->sP));
  TPM_HIP(hipStreamSynchronize(s->sE));
  s->release_planets();
  s->release_ring();
  s->ad.valid = false;
  s->mu0 = h.mu0;
  s->central_set = true;
  s->planets_set = false;
  s->particles_set = false;
  s->np = np;
  s->perm.assign(h.perm, h.perm + np);
  s->mu_s.assign(h.mu, h.mu + np);
  s->rcrit_s.assign(h.rcrit, h.rcrit + np);
  s->a_s.assign(h.a, h.a + np);
  const size_t b = sizeof(double) * 3 * std::max(np, 1);
  TPM_HIP(hipMalloc(&s->d_rj, b));
  TPM_HIP(hipMalloc(&s->d_vj, b));
  TPM_HIP(hipMalloc(&s->d_tmp, 4 * b));
  if (np > 0) {
    TPM_HIP(hipMemcpy(s->d_rj, h.rj, sizeof(double) * 3 * np, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(s->d_vj, h.vj, sizeof(double) * 3 * np, hipMemcpyHostToDevice));
  }
  TPM_HIP(hipMemcpy(s->d_flag, &h.flag, sizeof(int64_t), hipMemcpyHostToDevice));
  s->step = h.step;
  s->planets_set = true;
  s->rrem_set = false;
  return load_particles(s, n, r.data(), v.data(), step.data(), reason.data(), planet.data());
}

int tpm_get_stats(tpm_sim* s, tpm_stats* o) {
  if (!s || !o) return fail(TPM_EINVAL, "NULL argument");
  tpm_stats st = s->stats;
  st.sub_chunks = s->opt.sub_chunks;
  st.waves_per_simd = s->opt.waves_per_simd > 0 ? s->opt.waves_per_simd : s->last_wps;
  st.block_threads = s->opt.block_threads;
  st.chunk_steps = s->opt.chunk_steps;
  st.resync_chunks = s->opt.resync_chunks;
  st.step = s->step;
  st.n_particles = s->n;
  st.n_active = 0;
  for (int k = 0; k < 4; ++k) st.count_by_reason[k] = 0;
  if (s->particles_set && s->n > 0) {
    TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
    TPM_HIP(hipStreamSynchronize(s->sP));
    std::vector<int32_t> reason(s->n);
    TPM_HIP(launch_finalize(s->work[s->cur], s->d_nactive, s->n_active, s->out, s->sP));
    TPM_HIP(hipStreamSynchronize(s->sP));
    TPM_HIP(hipMemcpy(reason.data(), s->out.reason, s->n * 4, hipMemcpyDeviceToHost));
    for (auto x : reason)
      if (x >= 0 && x < 4) st.count_by_reason[x]++;
    st.n_active = st.count_by_reason[TPM_ACTIVE];
  }
  *o = st;
  return TPM_OK;
}

int tpm_planet_table(tpm_sim* s, int64_t nsteps, double dt, double* table) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "no planets");
  if (nsteps < 0 || !table) return fail(TPM_EINVAL, "bad arguments");
  if (!std::isfinite(dt) || dt == 0.0) return fail(TPM_EINVAL, "dt must be finite and non-zero");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  const int np = s->np, rl = 3 * np + 3;
  double *rj = nullptr, *vj = nullptr, *rows = nullptr;
  int64_t* flag = nullptr;
  size_t b = sizeof(double) * 3 * std::max(np, 1);
  TPM_HIP(hipStreamSynchronize(s->sE));
  DevScope mem;
  if (s->d_hist) {
    if (!s->hist_covers(s->step, nsteps, dt))
      return fail(TPM_EINVAL, "the rows' times leave the planet history");
    TPM_HIP(mem.alloc(rows, sizeof(double) * (nsteps + 1) * rl));
    TPM_HIP(launch_history_rows(s->hist(), rows, (int)(nsteps + 1), s->step, dt, nullptr, s->sE));
    std::vector<double> t((nsteps + 1) * rl);
    TPM_HIP(hipStreamSynchronize(s->sE));
    TPM_HIP(hipMemcpy(t.data(), rows, sizeof(double) * t.size(), hipMemcpyDeviceToHost));
    permute_table(s, t.data(), table, nsteps + 1, true);
    return TPM_OK;
  }
  TPM_HIP(mem.alloc(rj, b));
  TPM_HIP(mem.alloc(vj, b));
  TPM_HIP(mem.alloc(flag, sizeof(int64_t)));
  TPM_HIP(mem.alloc(rows, sizeof(double) * (nsteps + 1) * rl));
  TPM_HIP(hipMemcpy(rj, s->d_rj, b, hipMemcpyDeviceToDevice));
  TPM_HIP(hipMemcpy(vj, s->d_vj, b, hipMemcpyDeviceToDevice));
  int64_t m1 = -1;
  TPM_HIP(hipMemcpy(flag, &m1, sizeof(m1), hipMemcpyHostToDevice));
  const EphConst E = s->eph();
  const int K = s->opt.chunk_steps;
  for (int64_t c = 0; c * K < nsteps || c == 0; ++c) {
    int ks = (int)std::min<int64_t>(K, nsteps - c * K);
    TPM_HIP(launch_ephemeris_chunk(E, rj, vj, rows + (size_t)c * K * rl, ks, dt, s->step + c * K,
                                   flag, s->sE));
    if (nsteps == 0) break;
  }
  std::vector<double> t((nsteps + 1) * rl);
  TPM_HIP(hipStreamSynchronize(s->sE));
  TPM_HIP(hipMemcpy(t.data(), rows, sizeof(double) * t.size(), hipMemcpyDeviceToHost));
  int64_t f = -1;
  TPM_HIP(hipMemcpy(&f, flag, sizeof(f), hipMemcpyDeviceToHost));
  permute_table(s, t.data(), table, nsteps + 1, true);
  if (f == -2) return fail(TPM_EPLANET, "a planet orbit became unbound");
  if (f >= 0) return fail(TPM_EPLANET, "two planets came within a mutual Hill radius");
  return TPM_OK;
}

int tpm_debug_sincos(int64_t n, const double* x, double* s_out, double* c_out) {
  if (n < 0 || n >= (int64_t(1) << 31) || (n && (!x || !s_out || !c_out)))
    return fail(TPM_EINVAL, "bad arguments");
  if (n == 0) return TPM_OK;
  double *dx, *ds, *dc;
  DevScope mem;
  TPM_HIP(mem.alloc(dx, n * 8));
  TPM_HIP(mem.alloc(ds, n * 8));
  TPM_HIP(mem.alloc(dc, n * 8));
  TPM_HIP(hipMemcpy(dx, x, n * 8, hipMemcpyHostToDevice));
  TPM_HIP(launch_sincos_test(dx, ds, dc, (int)n, nullptr));
  TPM_HIP(hipDeviceSynchronize());
  TPM_HIP(hipMemcpy(s_out, ds, n * 8, hipMemcpyDeviceToHost));
  TPM_HIP(hipMemcpy(c_out, dc, n * 8, hipMemcpyDeviceToHost));
  return TPM_OK;
}

int tpm_debug_rsqrt(int64_t n, const double* x, double* out) {
  if (n < 0 || n >= (int64_t(1) << 31) || (n && (!x || !out)))
    return fail(TPM_EINVAL, "bad arguments");
  for (int64_t i = 0; i < n; ++i)
    if (!(x[i] > 0.0) || !std::isfinite(x[i])) return fail(TPM_EINVAL, "arguments must be finite and > 0");
  if (n == 0) return TPM_OK;
  double *dx, *dout;
  DevScope mem;
  TPM_HIP(mem.alloc(dx, n * 8));
  TPM_HIP(mem.alloc(dout, n * 5 * 8));
  TPM_HIP(hipMemcpy(dx, x, n * 8, hipMemcpyHostToDevice));
  TPM_HIP(launch_rsqrt_test(dx, dout, (int)n, nullptr));
  TPM_HIP(hipDeviceSynchronize());
  TPM_HIP(hipMemcpy(out, dout, n * 5 * 8, hipMemcpyDeviceToHost));
  return TPM_OK;
}

namespace {
int debug_drift(double mu, int64_t n, const double* rv_in, double* rv_out, int32_t* ok,
                double dt, int32_t kepler_iters, double kepler_ftol, int mode) {
  if (n < 0 || n >= (int64_t(1) << 31) || (n && (!rv_in || !rv_out || !ok)))
    return fail(TPM_EINVAL, "bad arguments");
  if (!(mu > 0.0) || !std::isfinite(dt) || kepler_iters < 0 || kepler_iters > 64)
    return fail(TPM_EINVAL, "bad arguments");
  if (n == 0) return TPM_OK;
  SysConst S{};
  S.mu0 = mu;
  S.inv_mu0 = 1.0 / mu;
  S.sqrt_mu0 = std::sqrt(mu);
  S.inv_sqrt_mu0 = 1.0 / std::sqrt(mu);
  S.kiters = kepler_iters;
  S.ftol = kepler_ftol > 0 ? kepler_ftol : 1e-13;
  S.universal = mode;
  double *di, *dout;
  int32_t* dok;
  DevScope mem;
  TPM_HIP(mem.alloc(di, n * 48));
  TPM_HIP(mem.alloc(dout, n * 48));
  TPM_HIP(mem.alloc(dok, n * 4));
  TPM_HIP(hipMemcpy(di, rv_in, n * 48, hipMemcpyHostToDevice));
  TPM_HIP(launch_drift_test(S, di, dout, dok, (int)n, dt, nullptr));
  TPM_HIP(hipDeviceSynchronize());
  TPM_HIP(hipMemcpy(rv_out, dout, n * 48, hipMemcpyDeviceToHost));
  TPM_HIP(hipMemcpy(ok, dok, n * 4, hipMemcpyDeviceToHost));
  return TPM_OK;
}
}  // namespace

int tpm_debug_drift(double mu, int64_t n, const double* rv_in, double* rv_out, int32_t* ok,
                    double dt, int32_t kepler_iters, double kepler_ftol) {
  return debug_drift(mu, n, rv_in, rv_out, ok, dt, kepler_iters, kepler_ftol, 0);
}

int tpm_debug_drift_universal(double mu, int64_t n, const double* rv_in, double* rv_out,
                              int32_t* ok, double dt, int32_t mode) {
  if (mode != 1 && mode != 2) return fail(TPM_EINVAL, "mode must be 1 or 2");
  return debug_drift(mu, n, rv_in, rv_out, ok, dt, 5, 0.0, mode);
}

}  // extern "C"

// ------------------------------------------------------------ derivatives
namespace {

template <class T>
int grow(T*& p, size_t& cap, size_t want) {
  if (cap >= want && p) return TPM_OK;
  dfree(p);
  TPM_HIP(hipMalloc(&p, sizeof(T) * std::max<size_t>(want, 1)));
  cap = want;
  return TPM_OK;
}

}  // namespace

extern "C" {

int tpm_ad_forward(tpm_sim* s, int64_t n, const double* d_r0, const double* d_v0, int64_t nsteps,
                   double dt, int32_t ckpt_every, double* d_rT, double* d_vT, int64_t* d_step,
                   int32_t* d_reason, void* stream) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  if (!s->planets_set) return fail(TPM_ESTATE, "set central mass and planets first");
  if (n < 0 || n >= (int64_t(1) << 31) || nsteps < 0 || nsteps >= (int64_t(1) << 31) ||
      ckpt_every <= 0)
    return fail(TPM_EINVAL, "bad sizes");
  if (n > 0 && (!d_r0 || !d_v0 || !d_rT || !d_vT)) return fail(TPM_EINVAL, "NULL array");
  if (!std::isfinite(dt) || dt == 0.0) return fail(TPM_EINVAL, "dt must be finite and non-zero");
  if (s->opt.handoff_substeps > 0)
    return fail(TPM_ESTATE, "derivatives of the close-encounter hand-off are not available");
  TPM_HIP(hipSetDevice(s->opt.device));
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  hipStream_t st = (hipStream_t)stream;
  auto& A = s->ad;
  A.valid = false;
  const int rl = 3 * s->np + 3;
  const int nseg = (int)((nsteps + ckpt_every - 1) / ckpt_every);
  size_t cap_n = A.cap_n;
  {
    int rc;
    if ((rc = grow(A.table, A.cap_table, (size_t)(nsteps + 1) * rl))) return rc;
    if ((rc = grow(A.ckpts, A.cap_ckpts, (size_t)(nseg + 1) * 6 * n))) return rc;
    if (cap_n < (size_t)n || !A.work) {
      dfree(A.work); dfree(A.dstep); dfree(A.reason); dfree(A.planet); dfree(A.treason);
      const size_t nn = std::max<size_t>(n, 1);
      TPM_HIP(hipMalloc(&A.work, sizeof(double) * 12 * nn));
      TPM_HIP(hipMalloc(&A.dstep, sizeof(int64_t) * nn));
      TPM_HIP(hipMalloc(&A.reason, sizeof(int32_t) * nn));
      TPM_HIP(hipMalloc(&A.planet, sizeof(int32_t) * nn));
      TPM_HIP(hipMalloc(&A.treason, sizeof(int32_t) * nn));
      A.cap_n = n;
    }
  }
  A.n = n;
  A.nsteps = nsteps;
  A.ckpt = ckpt_every;
  A.nseg = nseg;
  A.dt = dt;
  if (!A.ev_in) {
    for (int k = 0; k < 2; ++k) {
      TPM_HIP(hipEventCreateWithFlags(&A.ev_tab[k], hipEventDisableTiming));
      TPM_HIP(hipEventCreateWithFlags(&A.ev_rec[k], hipEventDisableTiming));
      TPM_HIP(hipEventCreateWithFlags(&A.ev_rev[k], hipEventDisableTiming));
    }
    TPM_HIP(hipEventCreateWithFlags(&A.ev_in, hipEventDisableTiming));
  }
  // The planet table of the whole run, from the current planet state (not
  // advanced), is computed on the library's planet-map stream in pieces of
  // whole segments (at least 1,024 steps), after whatever that stream already
  // holds (an earlier integrate); the caller's stream runs each segment once
  // the piece holding its last row is written, so the planet map and the
  // particle segments overlap.  A later tpm_integrate is ordered after these
  // pieces by the same stream.
  const SysConst S = s->sys();
  const EphConst E = s->eph();
  const size_t pb = sizeof(double) * 3 * std::max(s->np, 1);
  double* rj = s->d_tmp + 6 * std::max(s->np, 1);
  double* vj = rj + 3 * std::max(s->np, 1);
  TPM_HIP(hipMemcpyAsync(rj, s->d_rj, pb, hipMemcpyDeviceToDevice, s->sE));
  TPM_HIP(hipMemcpyAsync(vj, s->d_vj, pb, hipMemcpyDeviceToDevice, s->sE));
  TPM_HIP(launch_aos_to_soa(d_r0, d_v0, A.ckpts, n, st));
  const int64_t piece = (int64_t)ckpt_every * std::max<int64_t>(1, (1024 + ckpt_every - 1) / ckpt_every);
  int k = 0;   // next segment
  for (int64_t p0 = 0, j = 0;; p0 += piece, ++j) {
    const int64_t p1 = std::min<int64_t>(nsteps, p0 + piece);
    for (int64_t q0 = p0;;) {   // launches of at most 2^20 steps
      const int64_t q1 = std::min<int64_t>(p1, q0 + (int64_t(1) << 20));
      TPM_HIP(launch_ephemeris_chunk(E, rj, vj, A.table + (size_t)q0 * rl, (int)(q1 - q0), dt, q0,
                                     s->d_flag, s->sE));
      if ((q0 = q1) >= p1) break;
    }
    TPM_HIP(hipEventRecord(A.ev_tab[j % 2], s->sE));
    TPM_HIP(hipStreamWaitEvent(st, A.ev_tab[j % 2], 0));
    for (; k < nseg && std::min<int64_t>(nsteps, (int64_t)(k + 1) * ckpt_every) <= p1; ++k) {
      const int s0 = k * ckpt_every;
      const int s1 = (int)std::min<int64_t>(nsteps, (int64_t)s0 + ckpt_every);
      TPM_HIP(launch_ad_segment(S, dt, n, s0, s1, A.table, A.ckpts + (size_t)k * 6 * n,
                                A.ckpts + (size_t)(k + 1) * 6 * n, nullptr, A.dstep, A.reason,
                                A.planet, k == 0 ? 0 : 1, st));
    }
    if (p1 >= nsteps) break;
  }
  if (nseg == 0) {
    // no step: only the checks at step 0
    TPM_HIP(launch_ad_segment(S, dt, n, 0, 0, A.table, A.ckpts, nullptr, nullptr, A.dstep,
                              A.reason, A.planet, 0, st));
  }
  TPM_HIP(launch_soa_to_aos(A.ckpts + (size_t)nseg * 6 * n, d_rT, d_vT, n, st));
  if (d_step) TPM_HIP(hipMemcpyAsync(d_step, A.dstep, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
  if (d_reason) TPM_HIP(hipMemcpyAsync(d_reason, A.reason, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  A.valid = true;
  return TPM_OK;
}

int tpm_ad_backward(tpm_sim* s, const double* d_gRT, const double* d_gVT, double* d_gR0,
                    double* d_gV0, void* stream) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  auto& A = s->ad;
  if (!A.valid) return fail(TPM_ESTATE, "no tpm_ad_forward to differentiate");
  const int64_t n = A.n;
  if (n > 0 && (!d_gRT || !d_gVT || !d_gR0 || !d_gV0)) return fail(TPM_EINVAL, "NULL array");
  TPM_HIP(hipSetDevice(s->opt.device));
  hipStream_t st = (hipStream_t)stream;
  {
    int rc = grow(A.tape, A.cap_tape, (size_t)2 * A.ckpt * AD_TAPE_FIELDS * n);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> dev_lock(device_streams(s->opt.device).lock);
  const SysConst S = s->sys();
  double* lam = A.work;
  double* tape[2] = {A.tape, A.tape + (size_t)A.ckpt * AD_TAPE_FIELDS * n};
  // Segment k's states are recomputed from its checkpoint into tape k % 2 on
  // the library's particle stream while the caller's stream sweeps segment
  // k + 1 backwards through the other tape: the recomputation does not depend
  // on the adjoint, so the two overlap (each fills only part of the device at
  // these particle counts).  A recomputation waits until the sweep that last
  // read its tape is done; a sweep waits for its tape.
  const hipStream_t sR = s->sP;
  TPM_HIP(hipEventRecord(A.ev_in, st));
  TPM_HIP(hipStreamWaitEvent(sR, A.ev_in, 0));
  auto recompute = [&](int k) -> int {
    const int s0 = k * A.ckpt;
    const int s1 = (int)std::min<int64_t>(A.nsteps, (int64_t)s0 + A.ckpt);
    TPM_HIP(launch_ad_segment(S, A.dt, n, s0, s1, A.table, A.ckpts + (size_t)k * 6 * n, nullptr,
                              tape[k % 2], A.dstep, nullptr, nullptr, 2, sR));
    TPM_HIP(hipEventRecord(A.ev_rec[k % 2], sR));
    return TPM_OK;
  };
  TPM_HIP(launch_aos_to_soa(d_gRT, d_gVT, lam, n, st));
  for (int k = A.nseg - 1; k >= 0 && k >= A.nseg - 2; --k) {
    int rc = recompute(k);
    if (rc) return rc;
  }
  for (int k = A.nseg - 1; k >= 0; --k) {
    const int s0 = k * A.ckpt;
    const int s1 = (int)std::min<int64_t>(A.nsteps, (int64_t)s0 + A.ckpt);
    TPM_HIP(hipStreamWaitEvent(st, A.ev_rec[k % 2], 0));
    TPM_HIP(launch_ad_reverse(S, A.dt, n, s0, s1, A.table, tape[k % 2], lam, A.dstep, st));
    if (k >= 2) {
      TPM_HIP(hipEventRecord(A.ev_rev[k % 2], st));
      TPM_HIP(hipStreamWaitEvent(sR, A.ev_rev[k % 2], 0));
      int rc = recompute(k - 2);
      if (rc) return rc;
    }
  }
  // the library's stream is done with this call's tapes before anything else
  // runs on it
  TPM_HIP(hipEventRecord(A.ev_in, st));
  TPM_HIP(hipStreamWaitEvent(sR, A.ev_in, 0));
  TPM_HIP(launch_soa_to_aos(lam, d_gR0, d_gV0, n, st));
  return TPM_OK;
}

int tpm_ad_tangent(tpm_sim* s, const double* d_dR0, const double* d_dV0, double* d_dRT,
                   double* d_dVT, void* stream) {
  if (!s) return fail(TPM_EINVAL, "sim is NULL");
  auto& A = s->ad;
  if (!A.valid) return fail(TPM_ESTATE, "no tpm_ad_forward to differentiate");
  const int64_t n = A.n;
  if (n > 0 && (!d_dR0 || !d_dV0 || !d_dRT || !d_dVT)) return fail(TPM_EINVAL, "NULL array");
  TPM_HIP(hipSetDevice(s->opt.device));
  hipStream_t st = (hipStream_t)stream;
  const SysConst S = s->sys();
  double* state = A.work;
  double* tang = A.work + 6 * n;
  TPM_HIP(hipMemcpyAsync(state, A.ckpts, sizeof(double) * 6 * n, hipMemcpyDeviceToDevice, st));
  TPM_HIP(launch_aos_to_soa(d_dR0, d_dV0, tang, n, st));
  for (int k = 0; k < A.nseg; ++k) {
    const int s0 = k * A.ckpt;
    const int s1 = (int)std::min<int64_t>(A.nsteps, (int64_t)s0 + A.ckpt);
    TPM_HIP(launch_ad_tangent(S, A.dt, n, s0, s1, A.table, state, tang, A.treason, k == 0, st));
  }
  TPM_HIP(launch_soa_to_aos(tang, d_dRT, d_dVT, n, st));
  return TPM_OK;
}

}  // extern "C"

// ------------------------------------------------------------ many systems
// One call integrates nsys independent systems, each with its own central
// mass, planets (0..8), particles and time step, for the same number of
// steps.  The planet maps of all systems run as one launch per chunk (one
// wavefront each); the particles of all systems form one work queue whose
// tiles (64 particles of one system) are ordered by planet count, largest
// first.  The whole chunk loop is captured once into a HIP graph and launched
// once.  Every R chunks the graph compacts the working set (a stable
// partition keeps each system's survivors contiguous) and rebuilds the tiles
// on the device, so removed particles stop occupying lanes.  Workgroup size,
// chunk length and work-queue shape come from an autotuner that times one
// chunk of each candidate from the initial state; R from the measured cost of
// one compaction against a chunk's.  Choices are cached per (device, systems,
// particles, planet-count histogram, fixed options).
namespace {

struct BatchBuffers {
  EphConst* E = nullptr;
  SysDev* sys = nullptr;
  TileDesc* tiles = nullptr;
  double* rj = nullptr;
  double* vj = nullptr;
  double* dt = nullptr;
  int64_t* ring_off = nullptr;
  int64_t* flag = nullptr;
  double* ring = nullptr;
  Work w{};
  Work w2{};                  // second working set (compaction target)
  Out out{};
  int32_t* nall = nullptr;
  int32_t* psys = nullptr;    // [n] system of each particle (by slot)
  int32_t* sorder = nullptr;  // [nsys] systems in queue order
  int32_t* sbeg = nullptr;    // [nsys] scratch of the retiling
  int32_t* send = nullptr;
  int32_t* ntiles_dev = nullptr;
  int32_t* cscratch = nullptr;  // compaction scratch
  unsigned long long* ctr = nullptr;
  uint32_t* progress = nullptr;
  int32_t* qerr = nullptr;
  unsigned long long* acc = nullptr;
  // pristine copies for the autotuner's trial runs
  double* rj0 = nullptr;
  double* vj0 = nullptr;
  double* st0 = nullptr;
  ~BatchBuffers() {
    dfree(E); dfree(sys); dfree(tiles); dfree(rj); dfree(vj); dfree(dt); dfree(ring_off);
    dfree(flag); dfree(ring);
    for (Work* p : {&w, &w2}) {
      dfree(p->x); dfree(p->y); dfree(p->z); dfree(p->vx); dfree(p->vy); dfree(p->vz);
      dfree(p->slot); dfree(p->status);
    }
    dfree(psys); dfree(sorder); dfree(sbeg); dfree(send); dfree(ntiles_dev); dfree(cscratch);
    dfree(out.r); dfree(out.v); dfree(out.step); dfree(out.reason); dfree(out.planet);
    dfree(nall); dfree(ctr); dfree(progress); dfree(qerr); dfree(acc);
    dfree(rj0); dfree(vj0); dfree(st0);
  }
};

struct TuneChoice {
  int block, chunk, sub_chunks, waves_per_simd, resync;
};

std::map<std::string, TuneChoice>& tune_cache() {
  static std::map<std::string, TuneChoice> c;
  return c;
}

}  // namespace

extern "C" int tpm_batch_integrate(int32_t nsys, const double* mu0, const int32_t* planet_off,
                                   const double* mu_p, const double* rp, const double* vp,
                                   const double* rcrit, const int64_t* part_off, const double* r,
                                   const double* v, const double* dt, int64_t nsteps,
                                   const tpm_options* opt_in, double* r_out, double* v_out,
                                   int64_t* step_out, int32_t* reason_out, int32_t* planet_out,
                                   tpm_stats* stats_out, int64_t* planet_flag) {
  // ---- validation
  if (nsys <= 0 || !mu0 || !planet_off || !part_off || !dt) return fail(TPM_EINVAL, "bad arguments");
  if (nsteps < 0 || nsteps >= (int64_t(1) << 31)) return fail(TPM_EINVAL, "nsteps out of range");
  if (planet_off[0] != 0 || part_off[0] != 0) return fail(TPM_EINVAL, "offsets must start at 0");
  for (int s = 0; s < nsys; ++s) {
    const int np = planet_off[s + 1] - planet_off[s];
    if (np < 0 || np > MAX_NP) return fail(TPM_EINVAL, "planets per system must be 0..8");
    if (part_off[s + 1] < part_off[s]) return fail(TPM_EINVAL, "particle offsets must not decrease");
    if (!(std::isfinite(mu0[s]) && mu0[s] > 0.0)) return fail(TPM_EINVAL, "mu0 must be > 0");
    if (!std::isfinite(dt[s]) || dt[s] == 0.0) return fail(TPM_EINVAL, "dt must be finite and non-zero");
  }
  const int npl_total = planet_off[nsys];
  const int64_t n = part_off[nsys];
  if (n >= (int64_t(1) << 31)) return fail(TPM_EINVAL, "too many particles");
  if (npl_total > 0 && (!mu_p || !rp || !vp || !rcrit)) return fail(TPM_EINVAL, "NULL planet array");
  if (n > 0 && (!r || !v || !r_out || !v_out)) return fail(TPM_EINVAL, "NULL particle array");
  if (npl_total > 0 && !(finite_all(mu_p, npl_total) && finite_all(rp, 3 * npl_total) &&
                         finite_all(vp, 3 * npl_total) && finite_all(rcrit, npl_total)))
    return fail(TPM_EINVAL, "planet input not finite");
  if (n > 0 && !(finite_all(r, 3 * n) && finite_all(v, 3 * n)))
    return fail(TPM_EINVAL, "particle input not finite");
  tpm_options o;
  tpm_default_options(&o);
  if (opt_in) o = *opt_in;
  if (o.handoff_substeps != 0)
    return fail(TPM_EINVAL, "the close-encounter hand-off does not run in the many-system call");
  if (o.kepler_iters <= 0) o.kepler_iters = 5;
  if (o.chunk_steps < 0 || o.chunk_steps > (1 << 30)) return fail(TPM_EINVAL, "chunk_steps out of range");
  if (o.block_threads < 0 || o.block_threads % 64 || o.block_threads > 256)
    return fail(TPM_EINVAL, "bad block_threads");
  if (o.resync_chunks < 0) return fail(TPM_EINVAL, "resync_chunks < 0");
  if (!(o.kepler_ftol > 0.0)) o.kepler_ftol = 1e-13;
  // zero / negative members are the tuner's to choose
  const bool autotune = o.sub_chunks <= 0 || o.waves_per_simd <= 0 || o.chunk_steps == 0 ||
                        o.block_threads == 0 || o.resync_chunks == 0;
  static const int kChunks[] = {512, 1024, 2048};
  static const int kBlocks[] = {64, 256};
  const int Kmax = o.chunk_steps > 0 ? o.chunk_steps : 2048;

  // a device context via the single-system object (streams, events, device)
  tpm_options so = o;
  so.chunk_steps = Kmax;
  so.block_threads = 64;
  so.resync_chunks = 1;
  tpm_sim* ctx = nullptr;
  {
    int rc = tpm_create(&so, &ctx);
    if (rc) return rc;
  }
  std::unique_ptr<tpm_sim, void (*)(tpm_sim*)> guard(ctx, tpm_destroy);
  std::lock_guard<std::mutex> dev_lock(device_streams(o.device).lock);
  BatchBuffers B;
  const int64_t slot_rows = Kmax + 1;   // ring rows per slot (the longest candidate chunk)

  // ---- per-system set-up (host: ordering and constants; device: Jacobi)
  std::vector<EphConst> E(nsys);
  std::vector<SysDev> S(nsys);
  std::vector<std::vector<int>> perm(nsys);
  std::vector<double> hpos(3 * MAX_NP * nsys, 0.0), hvel(3 * MAX_NP * nsys, 0.0), dts(dt, dt + nsys);
  std::vector<int64_t> ring_off(nsys);
  int64_t ring_total = 0;
  int hist[MAX_NP + 1] = {0};
  for (int s = 0; s < nsys; ++s) {
    const int p0 = planet_off[s], np = planet_off[s + 1] - p0;
    std::vector<double> a;
    if (!sort_planets(mu0[s], np, mu_p + p0, rp + 3 * p0, vp + 3 * p0, perm[s], a))
      return fail(TPM_EINVAL, "planet orbit not bound in system " + std::to_string(s));
    std::vector<double> ms(np), as(np);
    SysDev& d = S[s];
    d = SysDev{};
    d.np = np;
    d.kiters = o.kepler_iters;
    d.ftol = o.kepler_ftol;
    d.rmax2 = o.r_escape > 0 ? o.r_escape * o.r_escape : INFINITY;
    d.dt = dt[s];
    d.K = KepConst{mu0[s], 1.0 / mu0[s], std::sqrt(mu0[s]), 1.0 / std::sqrt(mu0[s])};
    for (int j = 0; j < np; ++j) {
      const int c = perm[s][j];
      if (!(mu_p[p0 + c] > 0.0) || rcrit[p0 + c] < 0.0)
        return fail(TPM_EINVAL, "bad planet in system " + std::to_string(s));
      ms[j] = mu_p[p0 + c];
      as[j] = a[c];
      d.mu[j] = ms[j];
      d.rcrit2[j] = rcrit[p0 + c] * rcrit[p0 + c];
      for (int k = 0; k < 3; ++k) {
        hpos[3 * MAX_NP * s + 3 * j + k] = rp[3 * (p0 + c) + k];
        hvel[3 * MAX_NP * s + 3 * j + k] = vp[3 * (p0 + c) + k];
      }
    }
    E[s] = make_eph(mu0[s], np, ms.data(), as.data());
    ring_off[s] = ring_total;
    d.ring_off = ring_total;
    ring_total += (int64_t)NSLOT * slot_rows * (3 * np + 3);
    hist[np]++;
  }
  // tiles of 64 particles of one system, largest planet count first
  std::vector<TileDesc> tiles;
  for (int s = 0; s < nsys; ++s)
    for (int64_t f = part_off[s]; f < part_off[s + 1]; f += 64)
      tiles.push_back(TileDesc{s, (int32_t)f, (int32_t)std::min<int64_t>(64, part_off[s + 1] - f), 0});
  std::stable_sort(tiles.begin(), tiles.end(),
                   [&](const TileDesc& x, const TileDesc& y) { return S[x.sys].np > S[y.sys].np; });
  const int ntiles = (int)tiles.size();
  std::vector<int32_t> sorder(nsys), psys(std::max<int64_t>(n, 1), 0);
  std::iota(sorder.begin(), sorder.end(), 0);
  std::stable_sort(sorder.begin(), sorder.end(), [&](int x, int y) { return S[x].np > S[y].np; });
  for (int s = 0; s < nsys; ++s)
    for (int64_t i = part_off[s]; i < part_off[s + 1]; ++i) psys[i] = s;

  // ---- device buffers
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t ps = (size_t)3 * MAX_NP * nsys;
  TPM_HIP(hipMalloc(&B.E, sizeof(EphConst) * nsys));
  TPM_HIP(hipMalloc(&B.sys, sizeof(SysDev) * nsys));
  TPM_HIP(hipMalloc(&B.tiles, sizeof(TileDesc) * std::max(ntiles, 1)));
  TPM_HIP(hipMalloc(&B.rj, sizeof(double) * ps));
  TPM_HIP(hipMalloc(&B.vj, sizeof(double) * ps));
  TPM_HIP(hipMalloc(&B.rj0, sizeof(double) * ps));
  TPM_HIP(hipMalloc(&B.vj0, sizeof(double) * ps));
  TPM_HIP(hipMalloc(&B.dt, sizeof(double) * nsys));
  TPM_HIP(hipMalloc(&B.ring_off, sizeof(int64_t) * nsys));
  TPM_HIP(hipMalloc(&B.flag, sizeof(int64_t) * nsys));
  TPM_HIP(hipMalloc(&B.ring, sizeof(double) * std::max<int64_t>(ring_total, 1)));
  for (Work* W : {&B.w, &B.w2}) {
    for (double** p : {&W->x, &W->y, &W->z, &W->vx, &W->vy, &W->vz}) TPM_HIP(hipMalloc(p, nn * 8));
    TPM_HIP(hipMalloc(&W->slot, nn * 4));
    TPM_HIP(hipMalloc(&W->status, nn * 4));
  }
  TPM_HIP(hipMalloc(&B.psys, nn * 4));
  TPM_HIP(hipMalloc(&B.sorder, sizeof(int32_t) * nsys));
  TPM_HIP(hipMalloc(&B.sbeg, sizeof(int32_t) * nsys));
  TPM_HIP(hipMalloc(&B.send, sizeof(int32_t) * nsys));
  TPM_HIP(hipMalloc(&B.ntiles_dev, sizeof(int32_t)));
  TPM_HIP(hipMalloc(&B.cscratch, sizeof(int32_t) * compact_scratch_ints((int)nn)));
  TPM_HIP(hipMemcpy(B.psys, psys.data(), nn * 4, hipMemcpyHostToDevice));
  TPM_HIP(hipMemcpy(B.sorder, sorder.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice));
  TPM_HIP(hipMalloc(&B.out.r, nn * 24));
  TPM_HIP(hipMalloc(&B.out.v, nn * 24));
  TPM_HIP(hipMalloc(&B.out.step, nn * 8));
  TPM_HIP(hipMalloc(&B.out.reason, nn * 4));
  TPM_HIP(hipMalloc(&B.out.planet, nn * 4));
  TPM_HIP(hipMalloc(&B.st0, nn * 6 * 8));
  TPM_HIP(hipMalloc(&B.nall, sizeof(int32_t)));
  TPM_HIP(hipMalloc(&B.ctr, sizeof(unsigned long long)));
  TPM_HIP(hipMalloc(&B.progress, sizeof(uint32_t) * std::max(ntiles, 1)));
  TPM_HIP(hipMalloc(&B.qerr, sizeof(int32_t)));
  TPM_HIP(hipMalloc(&B.acc, sizeof(unsigned long long)));
  TPM_HIP(hipMemcpy(B.E, E.data(), sizeof(EphConst) * nsys, hipMemcpyHostToDevice));
  TPM_HIP(hipMemcpy(B.sys, S.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice));
  if (ntiles) TPM_HIP(hipMemcpy(B.tiles, tiles.data(), sizeof(TileDesc) * ntiles, hipMemcpyHostToDevice));
  TPM_HIP(hipMemcpy(B.dt, dts.data(), sizeof(double) * nsys, hipMemcpyHostToDevice));
  TPM_HIP(hipMemcpy(B.ring_off, ring_off.data(), sizeof(int64_t) * nsys, hipMemcpyHostToDevice));
  {
    std::vector<int64_t> m1(nsys, -1);
    TPM_HIP(hipMemcpy(B.flag, m1.data(), sizeof(int64_t) * nsys, hipMemcpyHostToDevice));
  }
  // planets: heliocentric -> Jacobi on the device (staged through rj0 / vj0)
  TPM_HIP(hipMemcpy(B.rj0, hpos.data(), sizeof(double) * ps, hipMemcpyHostToDevice));
  TPM_HIP(hipMemcpy(B.vj0, hvel.data(), sizeof(double) * ps, hipMemcpyHostToDevice));
  TPM_HIP(hipMemset(B.rj, 0, sizeof(double) * ps));
  TPM_HIP(hipMemset(B.vj, 0, sizeof(double) * ps));
  TPM_HIP(hipDeviceSynchronize());   // null-stream set-up before work on the non-blocking streams
  TPM_HIP(launch_helio_to_jacobi_batch(B.E, B.rj0, B.rj, nsys, ctx->sP));
  TPM_HIP(launch_helio_to_jacobi_batch(B.E, B.vj0, B.vj, nsys, ctx->sP));
  TPM_HIP(hipStreamSynchronize(ctx->sP));
  TPM_HIP(hipMemcpy(B.rj0, B.rj, sizeof(double) * ps, hipMemcpyDeviceToDevice));
  TPM_HIP(hipMemcpy(B.vj0, B.vj, sizeof(double) * ps, hipMemcpyDeviceToDevice));
  // particles: caller AoS -> SoA (global order = caller order)
  {
    std::vector<double> col(n);
    double* dst[6] = {B.w.x, B.w.y, B.w.z, B.w.vx, B.w.vy, B.w.vz};
    for (int c = 0; c < 6; ++c) {
      const double* src = c < 3 ? r : v;
      for (int64_t i = 0; i < n; ++i) col[i] = src[3 * i + (c % 3)];
      if (n) {
        TPM_HIP(hipMemcpy(dst[c], col.data(), n * 8, hipMemcpyHostToDevice));
        TPM_HIP(hipMemcpy(B.st0 + (size_t)c * n, col.data(), n * 8, hipMemcpyHostToDevice));
      }
    }
    std::vector<int32_t> idx(n), zero(n, 0);
    std::iota(idx.begin(), idx.end(), 0);
    if (n) {
      TPM_HIP(hipMemcpy(B.w.slot, idx.data(), n * 4, hipMemcpyHostToDevice));
      TPM_HIP(hipMemcpy(B.w.status, zero.data(), n * 4, hipMemcpyHostToDevice));
    }
  }
  const int32_t n32 = (int32_t)n;
  TPM_HIP(hipMemcpy(B.nall, &n32, 4, hipMemcpyHostToDevice));
  std::vector<int32_t> slot0(std::max<int64_t>(n, 1));
  std::iota(slot0.begin(), slot0.end(), 0);
  auto reset_run = [&]() -> int {
    // initial particle, planet and queue state (outside any captured graph)
    double* dst[6] = {B.w.x, B.w.y, B.w.z, B.w.vx, B.w.vy, B.w.vz};
    for (int c = 0; c < 6; ++c)
      if (n) TPM_HIP(hipMemcpy(dst[c], B.st0 + (size_t)c * n, n * 8, hipMemcpyDeviceToDevice));
    if (n) TPM_HIP(hipMemset(B.w.status, 0, n * 4));
    if (n) TPM_HIP(hipMemcpy(B.w.slot, slot0.data(), n * 4, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(B.nall, &n32, 4, hipMemcpyHostToDevice));
    if (ntiles) TPM_HIP(hipMemcpy(B.tiles, tiles.data(), sizeof(TileDesc) * ntiles, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(B.ntiles_dev, &ntiles, 4, hipMemcpyHostToDevice));
    TPM_HIP(hipMemcpy(B.rj, B.rj0, sizeof(double) * ps, hipMemcpyDeviceToDevice));
    TPM_HIP(hipMemcpy(B.vj, B.vj0, sizeof(double) * ps, hipMemcpyDeviceToDevice));
    TPM_HIP(hipMemset(B.ctr, 0, sizeof(unsigned long long)));
    TPM_HIP(hipMemset(B.progress, 0, sizeof(uint32_t) * std::max(ntiles, 1)));
    TPM_HIP(hipMemset(B.qerr, 0, sizeof(int32_t)));
    std::vector<int64_t> m1(std::max<int64_t>(n, nsys), -1);
    TPM_HIP(hipMemcpy(B.flag, m1.data(), sizeof(int64_t) * nsys, hipMemcpyHostToDevice));
    if (n) {
      TPM_HIP(hipMemcpy(B.out.step, m1.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice));
      TPM_HIP(hipMemset(B.out.reason, 0, n * 4));
    }
    TPM_HIP(hipDeviceSynchronize());
    return TPM_OK;
  };

  // ---- the chunk loop, enqueued on (sE: planet maps, sP: particles).  With
  // cfg.resync > 0 the working set is compacted after every resync-th chunk
  // (and the tiles rebuilt on the device); each particle launch then reads
  // its tile count from the device and starts from a zeroed item counter.
  // `cur` receives the working set holding the results.
  auto enqueue_run = [&](int64_t chunks, const TuneChoice& cfg, int& cur) -> int {
    const int K = cfg.chunk;
    unsigned long long base = 0;
    uint32_t epoch = 0;
    const int workers = std::max(1, std::min(ntiles, 4 * ctx->ncu * cfg.waves_per_simd));
    const int wpb = cfg.block / 64;
    const unsigned long long waves = (unsigned long long)((workers + wpb - 1) / wpb) * wpb;
    const bool compacting = cfg.resync > 0;
    Work ws[2] = {B.w, B.w2};
    cur = 0;
    TPM_HIP(hipEventRecord(ctx->ev_cnt[0], ctx->sP));
    TPM_HIP(hipStreamWaitEvent(ctx->sE, ctx->ev_cnt[0], 0));
    for (int64_t c = 0; c < chunks; ++c) {
      const int ks = (int)std::min<int64_t>(K, nsteps - c * K);
      const int slot = (int)(c % NSLOT);
      if (c >= NSLOT) TPM_HIP(hipStreamWaitEvent(ctx->sE, ctx->ev_done[slot], 0));
      TPM_HIP(launch_ephemeris_batch(B.E, B.rj, B.vj, B.ring, B.ring_off, slot, slot_rows, nsys, ks,
                                     B.dt, c * K, B.flag, ctx->sE));
      TPM_HIP(hipEventRecord(ctx->ev_eph[slot], ctx->sE));
      TPM_HIP(hipStreamWaitEvent(ctx->sP, ctx->ev_eph[slot], 0));
      BatchQueueArgs Q;
      Q.ctr = B.ctr;
      Q.base = compacting ? 0 : base;
      Q.progress = B.progress;
      Q.epoch = epoch;
      Q.ntiles = ntiles;
      Q.nsub = std::max(1, std::min(cfg.sub_chunks, ks));
      Q.sub_steps = (ks + Q.nsub - 1) / Q.nsub;
      Q.nsteps = ks;
      Q.step0 = c * (int64_t)K;
      Q.slot = slot;
      Q.slot_rows = slot_rows;
      Q.error = B.qerr;
      Q.ntiles_dev = compacting ? B.ntiles_dev : nullptr;
      if (compacting) TPM_HIP(launch_queue_reset(B.ctr, ctx->sP));
      TPM_HIP(launch_particle_batch(B.sys, B.tiles, ws[cur], B.out, B.ring, Q, workers, cfg.block,
                                    ctx->sP));
      if (ntiles > 0) {
        base += (unsigned long long)ntiles * Q.nsub + waves;
        epoch += (uint32_t)Q.nsub;
      }
      TPM_HIP(hipEventRecord(ctx->ev_done[slot], ctx->sP));
      if (compacting && (c + 1) % cfg.resync == 0 && c + 1 < chunks) {
        TPM_HIP(launch_compact(ws[cur], ws[1 - cur], B.nall, (int)n, B.cscratch, ctx->sP));
        cur = 1 - cur;
        TPM_HIP(launch_batch_retile(ws[cur], B.nall, (int)n, B.psys, B.sorder, nsys, B.sbeg, B.send,
                                    B.tiles, B.ntiles_dev, ctx->sP));
      }
    }
    TPM_HIP(hipEventRecord(ctx->ev_cnt[1], ctx->sE));
    TPM_HIP(hipStreamWaitEvent(ctx->sP, ctx->ev_cnt[1], 0));
    return TPM_OK;
  };

  // ---- autotuner: time one chunk of each (workgroup size, chunk length,
  // work-queue shape) candidate from the initial state, per step; then one
  // compaction, whose cost against the chosen chunk's sets the interval R
  // (compaction under 1% of the particle time)
  TuneChoice choice{o.block_threads > 0 ? o.block_threads : 64,
                    o.chunk_steps > 0 ? o.chunk_steps : 1024,
                    o.sub_chunks > 0 ? o.sub_chunks : 16, o.waves_per_simd > 0 ? o.waves_per_simd : 2,
                    o.resync_chunks > 0 ? o.resync_chunks : 1};
  int cur = 0;
  if (autotune && nsteps > 0 && ntiles > 0) {
    hipDeviceProp_t prop;
    TPM_HIP(hipGetDeviceProperties(&prop, o.device));
    std::string key = std::string(prop.gcnArchName) + "/" + std::to_string(nsys) + "/" +
                      std::to_string(n) + "/" + std::to_string(nsteps) + "/" +
                      std::to_string(o.block_threads) + "/" + std::to_string(o.chunk_steps) + "/" +
                      std::to_string(o.sub_chunks) + "/" + std::to_string(o.waves_per_simd) + "/" +
                      std::to_string(o.resync_chunks);
    for (int k = 0; k <= MAX_NP; ++k) key += "," + std::to_string(hist[k]);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      choice = it->second;
    } else {
      const int shapes[][2] = {{4, 2}, {8, 2}, {16, 2}, {4, 4}, {16, 4}};
      std::vector<TuneChoice> cands;
      for (int b : kBlocks) {
        if (o.block_threads > 0 && b != o.block_threads) continue;
        for (int k : kChunks) {
          if (o.chunk_steps > 0 && k != o.chunk_steps) continue;
          if (o.chunk_steps == 0 && k > std::max<int64_t>(512, nsteps)) continue;
          for (auto& sh : shapes) {
            if (o.sub_chunks > 0 && sh[0] != o.sub_chunks) continue;
            if (o.waves_per_simd > 0 && sh[1] != o.waves_per_simd) continue;
            cands.push_back(TuneChoice{b, k, sh[0], sh[1], 0});
          }
        }
      }
      if (o.block_threads > 0 && std::find(std::begin(kBlocks), std::end(kBlocks), o.block_threads) == std::end(kBlocks))
        for (auto& c : cands) c.block = o.block_threads;
      if (cands.empty()) cands.push_back(TuneChoice{choice.block, choice.chunk, choice.sub_chunks,
                                                    choice.waves_per_simd, 0});
      // time per step of `chunks` chunks of a candidate from the initial
      // state (the planet maps of the first chunk included)
      auto trial = [&](const TuneChoice& cand, int64_t chunks, double& per_step,
                       double& chunk_ms) -> int {
        int rc = reset_run();
        if (rc) return rc;
        TPM_HIP(hipEventRecord(ctx->t0P, ctx->sP));
        rc = enqueue_run(chunks, cand, cur);
        if (rc) return rc;
        TPM_HIP(hipEventRecord(ctx->t1P, ctx->sP));
        TPM_HIP(hipEventSynchronize(ctx->t1P));
        float ms = 0.f;
        TPM_HIP(hipEventElapsedTime(&ms, ctx->t0P, ctx->t1P));
        const int64_t steps = std::min<int64_t>(chunks * cand.chunk, nsteps);
        per_step = ms / (double)steps;
        chunk_ms = ms / (double)((steps + cand.chunk - 1) / cand.chunk);
        return TPM_OK;
      };
      // a screen of one chunk per candidate, then the best four again over
      // up to three chunks with a compaction after each (single-chunk times
      // differ by a few percent between neighbouring shapes, about the noise
      // of one launch)
      std::vector<std::pair<double, size_t>> screen;
      std::vector<double> chunk_ms_of(cands.size(), 0.0);
      for (size_t k = 0; k < cands.size(); ++k) {
        double ps = 0.0;
        int rc = trial(cands[k], 1, ps, chunk_ms_of[k]);
        if (rc) return rc;
        screen.emplace_back(ps, k);
      }
      std::sort(screen.begin(), screen.end());
      double best = 1e300, best_chunk_ms = 0.0;
      const size_t nfinal = std::min<size_t>(screen.size(), 4);
      for (size_t f = 0; f < nfinal; ++f) {
        TuneChoice cand = cands[screen[f].second];
        double ps = screen[f].first, cms = chunk_ms_of[screen[f].second];
        const int64_t nch = std::min<int64_t>(3, (nsteps + cand.chunk - 1) / cand.chunk);
        if (nfinal > 1 && nch > 1) {
          cand.resync = 1;
          int rc = trial(cand, nch, ps, cms);
          if (rc) return rc;
        }
        if (ps < best) {
          best = ps;
          best_chunk_ms = cms;
          const int keep_r = choice.resync;
          choice = cands[screen[f].second];
          choice.resync = keep_r;
        }
      }
      if (o.resync_chunks == 0) {
        int rc = reset_run();
        if (rc) return rc;
        TPM_HIP(hipEventRecord(ctx->t0P, ctx->sP));
        TPM_HIP(launch_compact(B.w, B.w2, B.nall, (int)n, B.cscratch, ctx->sP));
        TPM_HIP(launch_batch_retile(B.w2, B.nall, (int)n, B.psys, B.sorder, nsys, B.sbeg, B.send,
                                    B.tiles, B.ntiles_dev, ctx->sP));
        TPM_HIP(hipEventRecord(ctx->t1P, ctx->sP));
        TPM_HIP(hipEventSynchronize(ctx->t1P));
        float cms = 0.f;
        TPM_HIP(hipEventElapsedTime(&cms, ctx->t0P, ctx->t1P));
        choice.resync = std::max(1, (int)std::ceil(cms / (0.01 * std::max(best_chunk_ms, 1e-3))));
        choice.resync = std::min(choice.resync, 64);
      }
      tune_cache()[key] = choice;
    }
  }
  const int K = choice.chunk;
  const int64_t nchunks = (nsteps + K - 1) / K;

  // ---- capture the whole run into one graph and launch it once
  {
    int rc = reset_run();
    if (rc) return rc;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  TPM_HIP(hipStreamBeginCapture(ctx->sP, hipStreamCaptureModeThreadLocal));
  {
    int rc = enqueue_run(nchunks, choice, cur);
    if (rc) {
      (void)hipStreamEndCapture(ctx->sP, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
  }
  TPM_HIP(hipStreamEndCapture(ctx->sP, &graph));
  std::unique_ptr<std::remove_pointer<hipGraph_t>::type, hipError_t (*)(hipGraph_t)> gguard(
      graph, hipGraphDestroy);
  TPM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  std::unique_ptr<std::remove_pointer<hipGraphExec_t>::type, hipError_t (*)(hipGraphExec_t)> eguard(
      exec, hipGraphExecDestroy);
  auto w0 = std::chrono::steady_clock::now();
  TPM_HIP(hipEventRecord(ctx->t0P, ctx->sP));
  TPM_HIP(hipGraphLaunch(exec, ctx->sP));
  TPM_HIP(hipEventRecord(ctx->t1P, ctx->sP));
  TPM_HIP(hipStreamSynchronize(ctx->sP));
  auto w1 = std::chrono::steady_clock::now();
  float run_ms = 0.f;
  TPM_HIP(hipEventElapsedTime(&run_ms, ctx->t0P, ctx->t1P));
  {
    int32_t qerr = 0;
    TPM_HIP(hipMemcpy(&qerr, B.qerr, sizeof(qerr), hipMemcpyDeviceToHost));
    if (qerr) return fail(TPM_EDEVICE, "particle work queue: a wait exceeded its limit");
  }
  // ---- results
  TPM_HIP(launch_finalize(cur ? B.w2 : B.w, B.nall, (int)n, B.out, ctx->sP));
  TPM_HIP(hipMemsetAsync(B.acc, 0, sizeof(unsigned long long), ctx->sP));
  TPM_HIP(launch_active_steps(B.out.step, (int)n, 0, nsteps, B.acc, ctx->sP));
  TPM_HIP(hipStreamSynchronize(ctx->sP));
  if (n) {
    TPM_HIP(hipMemcpy(r_out, B.out.r, n * 24, hipMemcpyDeviceToHost));
    TPM_HIP(hipMemcpy(v_out, B.out.v, n * 24, hipMemcpyDeviceToHost));
    if (step_out) TPM_HIP(hipMemcpy(step_out, B.out.step, n * 8, hipMemcpyDeviceToHost));
    if (reason_out) TPM_HIP(hipMemcpy(reason_out, B.out.reason, n * 4, hipMemcpyDeviceToHost));
    if (planet_out) {
      TPM_HIP(hipMemcpy(planet_out, B.out.planet, n * 4, hipMemcpyDeviceToHost));
      for (int s = 0; s < nsys; ++s)
        for (int64_t i = part_off[s]; i < part_off[s + 1]; ++i)
          if (planet_out[i] >= 0) planet_out[i] = perm[s][planet_out[i]];
    }
  }
  unsigned long long acc = 0;
  TPM_HIP(hipMemcpy(&acc, B.acc, sizeof(acc), hipMemcpyDeviceToHost));
  std::vector<int64_t> flags(nsys);
  TPM_HIP(hipMemcpy(flags.data(), B.flag, sizeof(int64_t) * nsys, hipMemcpyDeviceToHost));
  if (stats_out) {
    tpm_stats st{};
    st.step = nsteps;
    st.n_particles = n;
    st.active_particle_steps = (int64_t)acc;
    st.wall_ms = std::chrono::duration<double, std::milli>(w1 - w0).count();
    st.particle_ms = run_ms;
    st.ephemeris_ms = run_ms;
    st.chunks = nchunks;
    st.sub_chunks = choice.sub_chunks;
    st.waves_per_simd = choice.waves_per_simd;
    st.block_threads = choice.block;
    st.chunk_steps = choice.chunk;
    st.resync_chunks = choice.resync;
    st.compactions = choice.resync > 0 ? (nchunks - 1) / choice.resync : 0;
    if (n) {
      std::vector<int32_t> rs(n);
      TPM_HIP(hipMemcpy(rs.data(), B.out.reason, n * 4, hipMemcpyDeviceToHost));
      for (auto x : rs)
        if (x >= 0 && x < 4) st.count_by_reason[x]++;
      st.n_active = st.count_by_reason[0];
    }
    *stats_out = st;
  }
  if (planet_flag) std::copy(flags.begin(), flags.end(), planet_flag);
  int nflag = 0, first = -1;
  for (int s = 0; s < nsys; ++s)
    if (flags[s] != -1) {
      if (first < 0) first = s;
      ++nflag;
    }
  if (nflag)
    return fail(TPM_EPLANET, std::to_string(nflag) + " system(s), first " + std::to_string(first) +
                                 ": planets came within a mutual Hill radius or a planet orbit "
                                 "became unbound");
  return TPM_OK;
}
