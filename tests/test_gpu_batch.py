"""Many systems in one graph launch (tpm_batch_integrate) on the GPU.

* bit-identical to running every system on its own (same kernels, same
  planet map, same per-particle arithmetic);
* parity with the oracle for sampled systems (1e-11 bar, identical removals);
* results independent of the work-queue shape (including the autotuner's);
* the full 512-system workload runs (reduced steps) with sampled parity.
"""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2011_03484_amd as P
    P.load()
    return P


def _single(P, w, T):
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    s.set_particles(w.r, w.v)
    s.integrate(T, w.dt)
    return s.particles()


def _systems(nsys=12, nmax=400, T=1000, seed=None):
    return W.make_batched(nsys=nsys, nmin=40, nmax=nmax, nsteps=T, seed=seed)


def test_batched_equals_per_system_runs(P):
    systems = _systems()
    T = 1000
    res, stats = P.batch_integrate(systems, nsteps=T, sub_chunks=4, waves_per_simd=2)
    assert sorted({w.np_ for w in systems}) == sorted(set(w.np_ for w in systems))
    removed = 0
    for w, g in zip(systems, res):
        ref = _single(P, w, T)
        for k in ("r", "v", "deact_step", "reason", "planet"):
            assert np.array_equal(g[k], ref[k]), (w.name, w.np_, k)
        removed += int(np.sum(g["reason"] != 0))
    print(f"systems {len(systems)}, Np set {sorted(set(w.np_ for w in systems))}, removed {removed}, "
          f"active particle-steps {stats['active_particle_steps']}", flush=True)


def test_batched_matches_oracle(P, orc):
    from test_gpu_parity import _compare, _oracle_reference
    systems = _systems(nsys=8, nmax=300, seed=77)
    T = 1000
    res, _ = P.batch_integrate(systems, nsteps=T)
    for w, g in zip(systems, res):
        eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, T, w.dt)
        ref, near, spread = _oracle_reference(orc, w.subset(nsteps=T), T, eph.table)
        _compare(g, ref, near, spread, f"batched/{w.name}/np{w.np_}")


def test_batched_shape_invariance(P):
    systems = _systems(nsys=10, nmax=300, seed=5)
    T = 600
    base, _ = P.batch_integrate(systems, nsteps=T, sub_chunks=1, waves_per_simd=1)
    for kw in ({"sub_chunks": 8, "waves_per_simd": 4}, {"sub_chunks": 3, "waves_per_simd": 2,
                                                       "chunk_steps": 128},
               {"block_threads": 256, "sub_chunks": 2, "waves_per_simd": 2},
               {"chunk_steps": 64, "resync_chunks": 1}, {"chunk_steps": 100, "resync_chunks": 3,
                                                         "block_threads": 128},
               {"chunk_steps": 512}, {}):
        other, st = P.batch_integrate(systems, nsteps=T, **kw)
        for a, b in zip(base, other):
            for k in ("r", "v", "deact_step", "reason", "planet"):
                assert np.array_equal(a[k], b[k]), (kw, k)
        print(f"{kw}: block {st['block_threads']} chunk {st['chunk_steps']} sub {st['sub_chunks']} "
              f"waves {st['waves_per_simd']} resync {st['resync_chunks']} "
              f"compactions {st['compactions']}", flush=True)
    assert st["sub_chunks"] > 0 and st["waves_per_simd"] > 0
    assert st["block_threads"] in (64, 256) and st["chunk_steps"] in (512, 1024, 2048)
    assert st["resync_chunks"] >= 1


def test_batched_compaction_with_heavy_removals(P):
    """Encounter radii ten times larger remove most particles within the first
    chunks; compacting after every 64-step chunk (the tiles rebuilt on the
    device inside the graph) gives every system bit for bit its own
    single-system result."""
    base = _systems(nsys=9, nmax=500, seed=21)
    T = 1000
    systems = [W.Workload(w.name, w.mu0, w.mu.copy(), w.rp.copy(), w.vp.copy(), 10 * w.rcrit,
                          w.rmax, w.r.copy(), w.v.copy(), w.dt, T) for w in base]
    res, st = P.batch_integrate(systems, nsteps=T, chunk_steps=64, resync_chunks=1, strict=False)
    removed = sum(int(np.sum(g["reason"] != 0)) for g in res)
    n = sum(w.n for w in systems)
    print(f"{removed} of {n} removed, {st['compactions']} compactions", flush=True)
    assert removed > n // 3 and st["compactions"] == (T + 63) // 64 - 1
    for w, g in zip(systems, res):
        ref = _single(P, w, T)
        for k in ("r", "v", "deact_step", "reason", "planet"):
            assert np.array_equal(g[k], ref[k]), (w.name, k)


def test_full_batched_workload_sampled(P, orc):
    """The 512-system workload (about 0.86M particles) for 2,000 steps; three
    systems checked against the oracle."""
    from test_gpu_parity import _compare, _oracle_reference
    systems = W.make_batched()
    T = 2000
    res, stats = P.batch_integrate(systems, nsteps=T)
    n = sum(w.n for w in systems)
    print(f"512 systems, {n} particles, {T} steps: graph {stats['particle_ms']:.1f} ms, "
          f"{stats['active_particle_steps'] / (stats['particle_ms'] / 1e3):.3e} particle-steps/s, "
          f"queue shape sub={stats['sub_chunks']} waves/SIMD={stats['waves_per_simd']}", flush=True)
    assert stats["active_particle_steps"] > 0.5 * n * T
    for idx in (0, 200, 511):
        w = systems[idx].subset(nsteps=T)
        eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, T, w.dt)
        ref, near, spread = _oracle_reference(orc, w, T, eph.table)
        _compare(res[idx], ref, near, spread, f"full/{w.name}/np{w.np_}")


def test_batched_edge_systems(P, orc):
    """A system with no planets, one with no particles, and one whose planets
    start inside a mutual Hill radius, alongside ordinary systems: only the
    close pair's system is flagged (at step 0, as in the oracle), every other
    system equals its own single-system run bit for bit, and the no-planet
    system matches the oracle."""
    import math
    from test_gpu_parity import _compare, _oracle_reference
    T = 500
    base = _systems(nsys=4, nmax=200, seed=9)
    w0 = base[1]
    noplanet = W.Workload("noplanet", w0.mu0, np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)),
                          np.zeros(0), w0.rmax, w0.r.copy(), w0.v.copy(), w0.dt, T)
    w1 = base[2]
    empty = W.Workload("empty", w1.mu0, w1.mu.copy(), w1.rp.copy(), w1.vp.copy(), w1.rcrit.copy(),
                       w1.rmax, np.zeros((0, 3)), np.zeros((0, 3)), w1.dt, T)
    mu0 = W.MU_SUN
    mu = np.array([1e-3, 1e-3]) * mu0
    rp, vp = W.elements_to_cartesian(mu0 + mu, np.array([5.0, 5.05]), np.zeros(2), np.zeros(2),
                                     np.zeros(2), np.zeros(2), np.array([0.0, 0.01]))
    rr = np.array([[20.0, 0, 0], [0, 25.0, 0]])
    vv = np.array([[0, math.sqrt(mu0 / 20.0), 0], [-math.sqrt(mu0 / 25.0), 0, 0]])
    pair = W.Workload("pair", mu0, mu, rp, vp, np.zeros(2), w0.rmax, rr, vv, 0.1, T)
    assert orc.ephemeris(mu0, mu, rp, vp, 10, 0.1).flag == 0
    # a planet set on a hyperbolic orbit (v^2 > 2 mu / r) is refused at set-up:
    # the Jacobi order needs every planet's semi-major axis
    hyp = W.Workload("hyperbolic", mu0, mu[:1].copy(), np.array([[5.0, 0, 0]]),
                     np.array([[0, 1.5 * math.sqrt(2 * (mu0 + mu[0]) / 5.0), 0]]), np.zeros(1),
                     w0.rmax, rr.copy(), vv.copy(), 0.1, T)
    with pytest.raises(P.TpmError, match="not bound in system 1"):
        P.batch_integrate([base[0], hyp], nsteps=10, strict=False)
    # two planets meeting at the line of nodes at step 412
    from test_oracle_pins import late_pair
    lm0, lmu, lrp, lvp, ldt, _, lfirst, _, _ = late_pair()
    late = W.Workload("late_pair", lm0, lmu, lrp, lvp, np.zeros(2), w0.rmax, rr.copy(), vv.copy(),
                      ldt, T)
    systems = [base[0], noplanet, base[1], empty, pair, base[2], base[3], late]
    res, stats = P.batch_integrate(systems, nsteps=T, strict=False)
    flags = stats["planet_flag"]
    # the pair is flagged at step 0 although its planets end up unbound later
    assert flags[4] == orc.ephemeris(mu0, mu, rp, vp, T, 0.1).flag == 0, flags
    assert flags[7] == orc.ephemeris(lm0, lmu, lrp, lvp, T, ldt).flag == lfirst, flags
    assert np.all(flags[[0, 1, 2, 3, 5, 6]] == -1), flags
    assert res[3]["r"].shape == (0, 3)
    for i in (0, 1, 2, 5, 6):
        ref = _single(P, systems[i], T)
        for k in ("r", "v", "deact_step", "reason", "planet"):
            assert np.array_equal(res[i][k], ref[k]), (systems[i].name, k)
    eph = orc.ephemeris(noplanet.mu0, noplanet.mu, noplanet.rp, noplanet.vp, T, noplanet.dt)
    ref, near, spread = _oracle_reference(orc, noplanet, T, eph.table)
    _compare(res[1], ref, near, spread, "batched/noplanet")
    with pytest.raises(P.PlanetEncounterError):
        P.batch_integrate(systems, nsteps=T)


def test_batched_backwards_equals_per_system_runs(P):
    """Negative steps (integration backwards in time) in the many-system call,
    mixed with forward systems: every system bit-identical to its own
    single-system run."""
    base = _systems(nsys=6, nmax=250, seed=13)
    T = 500
    systems = []
    for i, w in enumerate(base):
        dt = -w.dt if i % 2 == 0 else w.dt
        systems.append(W.Workload(w.name, w.mu0, w.mu.copy(), w.rp.copy(), w.vp.copy(), w.rcrit.copy(),
                                  w.rmax, w.r.copy(), w.v.copy(), dt, T))
    res, _ = P.batch_integrate(systems, nsteps=T)
    for w, g in zip(systems, res):
        ref = _single(P, w, T)
        for k in ("r", "v", "deact_step", "reason", "planet"):
            assert np.array_equal(g[k], ref[k]), (w.name, w.dt, k)
