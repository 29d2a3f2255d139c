/* tpmvs -- FP64 test-particle mixed-variable symplectic integrator for AMD
 * MI355X (gfx950).
 *
 * The method is that of Zhang & Gladman 2021 ("GLISSE", New Astronomy), sec. 2:
 * N massless test particles move in the field of a central mass m0 and Np
 * planets.  The planets are integrated once by the Wisdom-Holman map in Jacobi
 * coordinates (sec. 2.2, planet integration) and their heliocentric positions
 * plus the indirect term h0 = -sum_j mu_j r_j/|r_j|^3 are shared by every
 * particle (sec. 2.2).  Each particle step is a half kick
 *   dv/dt = h0 - sum_j mu_j (r - r_j)/|r - r_j|^3   (sec. 2.2, kick equation),
 * a Kepler drift about m0 for the full step solved by a fixed number of Newton
 * iterations of the difference form of Kepler's equation with f and g
 * functions (sec. 2.2), and a second half kick.  A particle is removed on close
 * approach to a planet (sec. 2.2, encounter criterion), on escape beyond
 * r_escape, or when its fixed-count Kepler solve does not converge (sec. 2.2),
 * and its state at that step boundary is kept.
 *
 * Conventions for every call:
 *  - Units are the caller's: mu = G m and dt must be consistent.
 *  - Vectors are row-major [n][3] float64 arrays (x, y, z), heliocentric.
 *  - The caller owns every buffer.  Inputs are copied before the call returns;
 *    outputs are written into caller buffers; no pointer is kept.
 *  - Return value: TPM_OK (0) or a negative TPM_E* code; tpm_last_error()
 *    then describes the failure.  Nothing is thrown or aborted across the ABI.
 *  - A tpm_sim is used by one host thread at a time.  All simulations on a
 *    device share that device's two library streams (created on first use,
 *    kept until the process ends); calls that enqueue work on them take a
 *    per-device lock, so calls from several threads on one device run one at
 *    a time.  The derivative calls (tpm_ad_backward, tpm_ad_tangent) run on
 *    the caller's stream.
 */
#ifndef TPMVS_H
#define TPMVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpm_sim tpm_sim;

enum {
  TPM_OK = 0,
  TPM_EINVAL = -1,   /* bad argument: NaN/Inf, size out of range, np > 8 ... */
  TPM_ENOMEM = -2,   /* device or host allocation failed                    */
  TPM_EDEVICE = -3,  /* HIP runtime error or no usable gfx950 device         */
  TPM_ESTATE = -4,   /* call out of order (e.g. integrate before set_*)      */
  TPM_EPLANET = -5   /* planets approached within a mutual Hill radius, or a
                        planet orbit became unbound: the planet map assumes no
                        planet-planet encounters (sec. 2.2).  The integration
                        was still carried out; results are returned.         */
};

/* Removal reasons (sec. 2.2, close-encounter and non-convergence paragraphs). */
enum {
  TPM_ACTIVE = 0,     /* still integrated                                   */
  TPM_ENCOUNTER = 1,  /* |r - r_j| < r_crit_j at a step boundary            */
  TPM_ESCAPE = 2,     /* |r| > r_escape at a step boundary                  */
  TPM_KEPLER = 3      /* unbound orbit, or |F(x_k)| > kepler_ftol after the
                         fixed kepler_iters Newton steps                      */
};

typedef struct {
  int32_t kepler_iters;   /* fixed Newton iterations per drift (sec. 2.2: five); default 5 */
  int32_t chunk_steps;    /* steps per particle launch ("planetary chunk", sec. 2.2); 0 = 8192.
                             When the planet map runs alongside the particles (no table
                             supplied), the first launch of each integrate call covers at
                             most 1,024 steps: the particles wait for its whole planet chunk */
  int32_t resync_chunks;  /* chunks between compactions ("resync interval", sec. 2.2); 0 = 1 */
  int32_t block_threads;  /* particle-kernel workgroup size (64..256, multiple of 64); 0 = 64 */
  int32_t sub_chunks;     /* work items per tile in a full chunk (dynamic load balance); a
                             shorter chunk gets proportionally fewer items of the same
                             length; 0 = 64 */
  int32_t waves_per_simd; /* particle wavefronts launched per SIMD (upper bound); 0 = as many
                             as the working set's tiles fill on every SIMD alike, 1..4,
                             chosen per launch */
  double r_escape;        /* remove when |r| > r_escape; <= 0 disables                */
  double kepler_ftol;     /* Kepler-failure threshold on |F(x_k)|; 0 = 1e-13         */
  int32_t device;         /* HIP device ordinal                                      */
  int32_t time_kernels;   /* 1: bracket every particle launch with HIP events        */
  /* High-eccentricity extensions of the Kepler step (sec. 2.2, Kepler-solver
   * paragraph, where the paper proposes them as future work):             */
  int32_t universal_drift;/* 1: a drift the fixed-iteration solve refuses (unbound or
                             near-parabolic orbit, |F(x_k)| > kepler_ftol) is taken in
                             universal variables instead, and the particle is removed
                             as TPM_KEPLER only if that gives no finite result; 0 = off.
                             It applies to tpm_integrate and the hand-off's encounter
                             integrator; tpm_integrate_static, tpm_batch_integrate and
                             the derivative calls (tpm_ad_*) take the fixed-iteration
                             drift alone, whatever this says.                       */
  int32_t sort_by_e;      /* 1: order the working set by decreasing osculating
                             eccentricity bin (bins of 0.1; unbound orbits first), so
                             wavefronts hold particles of similar Newton counts and the
                             most eccentric tiles are taken first; never changes
                             results; 0 = caller order                                */
  /* Close-encounter hand-off (sec. 5: particles in close encounters move off
   * the main integration; the paper leaves the method open, this library's
   * reading follows).  With handoff_substeps = M > 0, a particle that comes
   * within a planet's r_crit (tpm_set_planets; the hand-off radius) is not
   * removed but handed off to a secondary kernel that integrates the list of
   * such particles behind the main kernel, on a stream of its own (the call
   * keeps all its planet rows for it: (chunk_steps + 1) x (6 Np + 3) x 8
   * bytes per chunk; a call needing more than 4 GiB, or than the environment
   * variable TPM_HANDOFF_RING_BYTES says, runs as several, with no change of
   * result):
   * at every step boundary a particle within the hand-off radius of any
   * planet takes its next step as M equal substeps of the same kick - drift -
   * kick, with the planets between the two table rows on the cubic Hermite
   * interpolant of their heliocentric positions and velocities (the row
   * values at the step's two ends) and h0 from the interpolated positions;
   * any other step is the plain map step.  A particle is removed within its
   * removal radius (tpm_set_removal_radii) at any step or substep boundary
   * (reason TPM_ENCOUNTER; step n at a step boundary, n + 1 at a substep
   * inside step n, keeping that substep's state), beyond r_escape at a step
   * boundary, or on a refused drift (TPM_KEPLER, the state at the start of
   * the failing substep).  The list's particles rejoin the main working set
   * at the end of each tpm_integrate.  Needs the on-device planet map (no
   * supplied table or history) and removal radii; tpm_integrate returns
   * TPM_ESTATE otherwise, and with diagnostics on.  The derivative, many-system
   * and no-allocation calls refuse it.  0 = off (removal at r_crit).          */
  int32_t handoff_substeps;
} tpm_options;

typedef struct {
  int64_t step;                   /* global step reached                          */
  int64_t n_particles;
  int64_t n_active;               /* particles still active                       */
  int64_t active_particle_steps;  /* particle-steps done while active, last integrate */
  double wall_ms;                 /* last integrate, host wall clock incl. sync   */
  double particle_ms;             /* last integrate, HIP events on the particle stream */
  double ephemeris_ms;            /* last integrate, HIP events on the ephemeris stream */
  int64_t chunks;                 /* particle launches in the last integrate      */
  double particle_kernel_ms;      /* last integrate, sum of HIP-event durations of the
                                     particle launches alone (only with time_kernels) */
  int64_t compactions;            /* compactions in the last integrate            */
  int64_t count_by_reason[4];     /* over all particles                           */
  int32_t sub_chunks;             /* work-queue shape used (after autotuning)     */
  int32_t waves_per_simd;
  int32_t block_threads;          /* workgroup size, chunk length and compaction  */
  int32_t chunk_steps;            /* interval used (after autotuning)             */
  int32_t resync_chunks;
  int64_t handoffs;               /* close-encounter hand-offs in the last integrate */
} tpm_stats;

/* Fill *opt with the defaults listed above. */
void tpm_default_options(tpm_options* opt);

/* Create a simulation on opt->device (opt may be NULL for defaults).
 * TPM_EDEVICE if the device cannot be used. */
int tpm_create(const tpm_options* opt, tpm_sim** out);
void tpm_destroy(tpm_sim* sim);

/* Central mass mu0 = G m0 > 0.  Must precede tpm_set_planets. */
int tpm_set_central(tpm_sim* sim, double mu0);

/* np (0..8) planets: mu[np] = G m_j > 0, heliocentric r[np][3], v[np][3], and
 * the encounter radius r_crit[np] >= 0 of each (a fixed distance or a Hill
 * multiple, sec. 2.2; see tpm_hill_radius).  Planets may be given in any order;
 * they are integrated sorted by osculating semi-major axis (the Jacobi order of
 * sec. 2.2) but every output uses the caller's order.  Resets the step count.
 * TPM_EINVAL if a planet's osculating orbit about mu0 + mu_j is not bound
 * (its semi-major axis fixes the order and the mutual Hill limits). */
int tpm_set_planets(tpm_sim* sim, int32_t np, const double* mu, const double* r,
                    const double* v, const double* r_crit);

/* n particles, heliocentric r[n][3], v[n][3]; all active.  0 <= n < 2^31. */
int tpm_set_particles(tpm_sim* sim, int64_t n, const double* r, const double* v);

/* Removal radii r_rem[np] (> 0, caller planet order) of the close-encounter
 * hand-off (see tpm_options.handoff_substeps): a handed-off particle within
 * r_rem of a planet is removed.  After tpm_set_planets (which, like
 * tpm_set_state, clears them); TPM_ESTATE before it, TPM_EINVAL for a radius
 * that is not positive and finite. */
int tpm_set_removal_radii(tpm_sim* sim, const double* r_rem);

/* Advance planets and particles by nsteps steps of dt (dt < 0 integrates
 * backwards).  Checks run at every step boundary, including the first and last.
 * Calling it twice with T1 and T2 steps gives bit-identical results to one call
 * with T1 + T2 steps, and so does a new simulation set from tpm_get_state
 * (tpm_set_state).  Resuming instead from tpm_get_planets and the still-active
 * particles of tpm_get_particles (step count restarting at 0) agrees with the
 * uninterrupted run to rounding: the planets' Jacobi state passes through
 * heliocentric coordinates once more.  TPM_EINVAL and TPM_ESTATE are returned
 * before any work is enqueued and leave the simulation as it was; after
 * TPM_ENOMEM or TPM_EDEVICE
 * the integration stopped part-way and the simulation's state is undefined
 * (destroy it). */
int tpm_integrate(tpm_sim* sim, int64_t nsteps, double dt);

/* Particle results in the caller's order (any pointer may be NULL): r, v [n][3]
 * (removed particles keep the state of their removal step), deact_step[n]
 * (-1 while active), reason[n] (TPM_ACTIVE...), planet[n] (caller index of the
 * planet for TPM_ENCOUNTER, else -1). */
int tpm_get_particles(tpm_sim* sim, double* r, double* v, int64_t* deact_step,
                      int32_t* reason, int32_t* planet);

/* Current heliocentric planet state, caller order, r[np][3], v[np][3]. */
int tpm_get_planets(tpm_sim* sim, double* r, double* v);

int tpm_get_stats(tpm_sim* sim, tpm_stats* out);

/* ---- state of a simulation, for checkpoints and continuation runs ----------
 * The paper continues integrations from their output states (sec. 4.2); these
 * carry the whole internal state, so a continuation is bit-identical to the
 * uninterrupted run.  tpm_get_state writes an opaque blob into caller memory:
 * the central mass, the planets (constants, their integration order and the
 * Jacobi state the planet map carries), the global step count, the first
 * planet event so far, and every particle's state and removal record.  With
 * buf NULL it only stores the blob's size in *size; otherwise *size is the
 * buffer's capacity on entry (TPM_EINVAL if too small) and the blob's size on
 * return.  TPM_ESTATE before planets and particles are set.
 * tpm_set_state replaces the central mass, planets, particles, step count and
 * planet event of sim (created with any options) by those of a blob of exactly
 * `size` bytes from this library version (TPM_EINVAL otherwise, before
 * anything changes).  Integrating after it continues the run: removal steps
 * stay absolute, and the results equal those of one uninterrupted run bit for
 * bit.  A caller-supplied planet table and the derivative context are
 * dropped.  The blob is native-endian and meant for the same library. */
int tpm_get_state(tpm_sim* sim, void* buf, int64_t* size);
int tpm_set_state(tpm_sim* sim, const void* buf, int64_t size);

/* ---- sampled diagnostics and snapshots ---------------------------------------
 * The paper's applications read orbital elements logged at a fixed interval
 * (sec. 4.2: every 2,048 yr) and its integrator copies the particle arrays
 * back to the host after a configurable number of chunks for periodic output
 * (sec. 2.2).  With diagnostics on, every global step boundary that is a
 * multiple of `every` (a particle launch ends there; the first boundary of an
 * integrate call is sampled too unless it already was) samples each particle
 * that is active there and passes that boundary's removal test:
 *  - its osculating heliocentric eccentricity about mu0, keeping the largest
 *    and the first sampled step that reached it (sec. 3.3);
 *  - for each of nres (0..2) resonances p:q with the reference planet, the
 *    resonant angle phi = p lambda - q lambda_ref - (p - q) varpi (sec. 4.1;
 *    lambda mean longitude, varpi longitude of pericentre, the planet's
 *    elements about mu0 + mu_ref).  flags[i][k] bit 0 records a sample with
 *    phi within 10 degrees of 0, bit 1 one within 10 degrees of 180 degrees;
 *    the paper's libration criterion (sec. 4.2: never within 10 degrees of one
 *    of them) holds unless both bits are set.  phi_lo/phi_hi[i][k] bound
 *    phi - 180 degrees, folded into (-180, 180] degrees (radians).
 * A snapshot callback (may be NULL) receives, at each sample, every particle
 * in the caller's order: r, v [n][3]; deact_step, reason as in
 * tpm_get_particles (a particle removed at the sample's own step shows its
 * removal); its osculating elements [n][6] (a, e, inc, node, peri, M about
 * mu0, radians; from the removal state for removed particles).  The arrays
 * live in library memory, valid during the call only.  It runs on the thread
 * inside tpm_integrate, in step order, at most two samples behind the GPU,
 * and must not call the library.
 * Resonant angles need the planets' velocities: with a supplied planet table
 * tpm_integrate returns TPM_ESTATE.  tpm_set_diagnostics (after planets and
 * particles; every = 0 or opt NULL turns it off) starts the accumulators
 * afresh: e_max -1, its step -1, flags 0, phi_lo +inf, phi_hi -inf.
 * tpm_set_planets, tpm_set_particles and tpm_set_state turn diagnostics off.
 * The batched and no-allocation entry points do not sample. */
typedef void (*tpm_snapshot_fn)(void* user, int64_t step, int64_t n, const double* r,
                                const double* v, const int64_t* deact_step,
                                const int32_t* reason, const double* elements);
typedef struct {
  int64_t every;          /* sample interval in steps (> 0); 0 = off                 */
  int32_t ref_planet;     /* caller index of the resonances' planet                  */
  int32_t nres;           /* 0..2                                                    */
  int32_t p[2], q[2];     /* resonance k is p[k]:q[k] (e.g. 3:1, 5:2 with Neptune)   */
  tpm_snapshot_fn snapshot;
  void* user;             /* passed to snapshot                                      */
} tpm_diag_options;
int tpm_set_diagnostics(tpm_sim* sim, const tpm_diag_options* opt);
/* emax[n], emax_step[n], flags[n][nres], phi_lo[n][nres], phi_hi[n][nres]
 * (caller order; any may be NULL).  TPM_ESTATE when diagnostics are off. */
int tpm_get_diagnostics(tpm_sim* sim, double* emax, int64_t* emax_step, int32_t* flags,
                        double* phi_lo, double* phi_hi);

/* Hill radius a_p (mu_p / (3 mu0))^(1/3) (sec. 2.2, encounter criterion). */
double tpm_hill_radius(double mu0, double mu_p, double a_p);

/* Message of the last failing call on this thread ("" if none). */
const char* tpm_last_error(void);

/* ---- planet table ---------------------------------------------------------
 * Run the planet map from the current planet state for nsteps steps of dt and
 * write the table rows [nsteps+1][3np+3] (r_1..r_np heliocentric in the
 * caller's planet order, then h0) to host memory.  The simulation state is not
 * advanced.  Returns TPM_EPLANET under the same condition as tpm_integrate. */
int tpm_planet_table(tpm_sim* sim, int64_t nsteps, double dt, double* table);

/* Use a caller-supplied planet table (rows [nrows][3np+3], same layout, row n =
 * global step n) instead of the on-device planet map, from now on; nrows <= 0
 * returns to the planet map.  Meant for checking the particle kernel alone. */
int tpm_set_planet_table(tpm_sim* sim, const double* table, int64_t nrows);

/* Take the planet positions from a history instead of the on-device planet map
 * (sec. 2.2: they may come from any source, such as interpolation from a
 * history file), from now on.  nrec records at strictly increasing times
 * t[nrec] hold heliocentric planet positions r[nrec][np][3] and velocities
 * v[nrec][np][3] (caller planet order, as in tpm_set_planets; host arrays,
 * copied).  Row n of every run (global step n) lies at time t0 + n dt; each
 * planet there follows the cubic Hermite interpolant of the two records around
 * that time (matching both positions and both velocities), and h0 is computed
 * from the interpolated positions.  The rows of each chunk are interpolated on
 * the device, one thread per row.  tpm_integrate returns TPM_EINVAL (before any
 * work) if a row's time leaves [t[0], t[nrec-1]]; tpm_get_planets returns the
 * interpolated state at the current step; tpm_planet_table the interpolated
 * rows.  No planet-planet test runs (the planets are not integrated).  nrec <= 0
 * returns to the planet map (its state is where tpm_set_planets left it).  It
 * replaces a supplied planet table and vice versa. */
int tpm_set_planet_history(tpm_sim* sim, int64_t nrec, const double* t, const double* r,
                           const double* v, double t0);

/* ---- derivatives of the particle map ---------------------------------------
 * Device-pointer calls for autograd frameworks: every array is caller-owned
 * device memory, [n][3] row-major float64 unless stated; work is enqueued on
 * the caller's HIP stream `stream` (NULL = null stream) without synchronising,
 * so outputs are ready when that stream reaches them.  The planets are not
 * differentiated.  A removed particle keeps the state of its removal step, so
 * its derivative is that of the map up to that step.
 *
 * tpm_ad_forward: integrates n particles from (d_r0, d_v0) for nsteps steps of
 * dt through the planets set on sim (their state is not advanced) and writes
 * d_rT, d_vT, d_step[n] (int64, removal step or -1) and d_reason[n] (int32)
 * (those two may be NULL).  It keeps, inside sim, the planet table of the run
 * and the particle states every ckpt_every steps; they are the context of the
 * next tpm_ad_backward / tpm_ad_tangent (one context per sim: a new forward
 * replaces it).
 * tpm_ad_backward: vector-Jacobian product (dL/dr_0, dL/dv_0) from
 * (dL/dr_T, dL/dv_T): each segment of ckpt_every steps is recomputed from its
 * checkpoint into a tape of ckpt_every x 96 n bytes (per particle and step: the
 * state, the opening kick's acceleration and the drift's Kepler root), and
 * swept backwards; the library holds two such tapes.
 * tpm_ad_tangent: Jacobian-vector product (d r_T, d v_T) from (d r_0, d v_0)
 * for the run of the last forward.
 * TPM_ESTATE if no forward has been run. */
int tpm_ad_forward(tpm_sim* sim, int64_t n, const double* d_r0, const double* d_v0,
                   int64_t nsteps, double dt, int32_t ckpt_every, double* d_rT, double* d_vT,
                   int64_t* d_step, int32_t* d_reason, void* stream);
int tpm_ad_backward(tpm_sim* sim, const double* d_gRT, const double* d_gVT, double* d_gR0,
                    double* d_gV0, void* stream);
int tpm_ad_tangent(tpm_sim* sim, const double* d_dR0, const double* d_dV0, double* d_dRT,
                   double* d_dVT, void* stream);

/* ---- many systems in one launch ---------------------------------------------
 * nsys independent systems (central mass, 0..8 planets, particles, own time
 * step) advanced by the same number of steps.  Host arrays; CSR-style offsets:
 * system s has planets planet_off[s]..planet_off[s+1]-1 (mu_p, rp[.][3],
 * vp[.][3], rcrit) and particles part_off[s]..part_off[s+1]-1 (r[.][3],
 * v[.][3]); mu0[s], dt[s].  Outputs as in tpm_get_particles (planet indices
 * local to the particle's system, caller order).  r_escape, kepler_iters,
 * kepler_ftol and device come from opt (NULL = defaults).  block_threads,
 * chunk_steps, sub_chunks, waves_per_simd and resync_chunks that are 0 are
 * chosen by an autotuner: it times one chunk of each candidate (workgroup size
 * 64 or 256, chunk length 512, 1,024 or 2,048 steps, five work-queue shapes)
 * from the initial state, per step, and sets the compaction interval so that
 * one compaction costs under 1% of the chunks it follows; choices are cached
 * per (device, systems, particles, steps, planet-count histogram, fixed
 * options) and never change results.  The planet maps of all systems run as
 * one launch per chunk and the particles of all systems as one work queue
 * (tiles of 64 particles of one system, most planets first); every
 * resync_chunks chunks the working set is compacted and the tiles rebuilt on
 * the device.  The whole run is captured into one HIP graph and launched once.
 * stats (may be NULL) receives the graph's run time, the active
 * particle-steps and the chosen shape.  planet_flag (may be NULL) receives per system
 * the first of these events: -1 none, t >= 0 two planets within a mutual
 * Hill radius at step t, -2 a planet orbit found unbound in a drift (before
 * any close pair; it wins a tie with a pair seen at the end of the same step).
 * Any flag makes the call return TPM_EPLANET; the run goes on and all results
 * are still written.  A system whose planets are not all bound at the start is
 * refused with TPM_EINVAL, as in tpm_set_planets. */
int tpm_batch_integrate(int32_t nsys, const double* mu0, const int32_t* planet_off,
                        const double* mu_p, const double* rp, const double* vp,
                        const double* rcrit, const int64_t* part_off, const double* r,
                        const double* v, const double* dt, int64_t nsteps,
                        const tpm_options* opt, double* r_out, double* v_out, int64_t* step_out,
                        int32_t* reason_out, int32_t* planet_out, tpm_stats* stats,
                        int64_t* planet_flag);

/* ---- one run without allocation ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One call does
 * what tpm_set_central, tpm_set_planets, tpm_set_particles, tpm_integrate and
 * tpm_get_particles do on a new simulation, with the same kernels and bit-
 * identical results, but it allocates nothing: every buffer the kernels need
 * beyond the inputs and outputs (working set, planet-table rows, work-queue
 * counters, compaction scratch, planet state) lies in one fixed device array
 * of the library (about 30 MiB, held by each GPU the library runs on until the
 * process ends).  Limits: n <= 262,144 particles, chunk_steps <= 8192 (0 =
 * 8192), np <= 8; larger requests return TPM_EINVAL before any work.
 * Planets (mu[np], rp[np][3], vp[np][3], rcrit[np]) are host arrays, read
 * before the call returns.  d_r, d_v [n][3] (input) and d_r_out, d_v_out
 * [n][3], d_step[n] (int64), d_reason[n], d_planet[n] (int32) (outputs, as in
 * tpm_get_particles) are caller-owned device memory; d_info (device, 2 int64,
 * may be NULL) receives the planet event (-1 none, t >= 0 two planets within a
 * mutual Hill radius at step t, -2 a planet orbit found unbound) and the
 * work-queue error flag (0 = none).  Work is enqueued on the caller's stream
 * (NULL = null stream) without synchronising; options as in tpm_create (NULL =
 * defaults; time_kernels is ignored).  The planet map and the particles run one
 * after the other on that one stream, so a run takes about the sum of the two
 * stages rather than the larger.  Every call on one GPU uses that GPU's array,
 * which keeps the last call's contents (each call initialises what it uses):
 * calls that overlap on one GPU, from any stream or thread, race. */
int tpm_integrate_static(const tpm_options* opt, double mu0, int32_t np, const double* mu,
                         const double* rp, const double* vp, const double* rcrit, int64_t n,
                         const double* d_r, const double* d_v, int64_t nsteps, double dt,
                         double* d_r_out, double* d_v_out, int64_t* d_step, int32_t* d_reason,
                         int32_t* d_planet, int64_t* d_info, void* stream);

/* ---- unit entry points of the device math (host arrays) -------------------- */
/* sin and cos of x[n] by the library's branch-free FP64 routine. */
int tpm_debug_sincos(int64_t n, const double* x, double* s, double* c);
/* The library's FP64 reciprocal square root and its relatives, for x[n]
 * finite and > 0 (else TPM_EINVAL): out[5 i + k] holds, for k = 0..4,
 * 1/sqrt(x), sqrt(x), 1/x, x^(-3/2) and x^(-3/2) to about 2^-45 (the
 * perturbation kick's factor).  out holds 5 n doubles; both arrays are host
 * memory owned by the caller. */
int tpm_debug_rsqrt(int64_t n, const double* x, double* out);
/* One fixed-iteration Kepler drift about mu of each rv[n][6] (x, y, z, vx, vy,
 * vz) by dt; ok[n] = 0 where the drift was refused (TPM_KEPLER rule). */
int tpm_debug_drift(double mu, int64_t n, const double* rv_in, double* rv_out, int32_t* ok,
                    double dt, int32_t kepler_iters, double kepler_ftol);
/* The universal-variable drift (see tpm_options.universal_drift) of each
 * rv[n][6] by dt about mu: mode 1 as the particle kernel takes it (the five-
 * iteration solve first, the universal drift where that is refused), mode 2
 * the universal drift alone; ok[n] = 0 where no finite result was reached
 * (rv_out then holds the input state).  Host arrays. */
int tpm_debug_drift_universal(double mu, int64_t n, const double* rv_in, double* rv_out,
                              int32_t* ok, double dt, int32_t mode);

#ifdef __cplusplus
}
#endif

#endif /* TPMVS_H */
