"""GPU parity of the close-encounter hand-off (sec. 5; the reading is stated in
the oracle above run_particle_handoff and in include/tpmvs.h): particles that
come within a planet's hand-off radius move from the main kernel to the
encounter list, which a secondary kernel integrates one chunk behind.

  * with one substep an encounter step is the plain map step, so the run
    equals the plain run with the removal radius as its encounter radius, bit
    for bit (both on the GPU);
  * against the oracle: removal records identical and states within the
    parity bar of tests/test_gpu_parity.py (plain 1e-11 for regular
    particles, 100 x the oracle's spread for chaotic ones), where a
    particle's spread here also covers the encounter phase: the oracle's
    response to a one-ulp change of its start and of the first planet's, and
    to its contracted build;
  * splitting a run over several calls changes nothing, bit for bit;
  * the calls that cannot run it refuse it.
"""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W
from test_gpu_parity import _compare

pytestmark = pytest.mark.gpu

KEYS = ("r", "v", "deact_step", "reason", "planet")


@pytest.fixture(scope="module")
def tpm():
    import paper_2011_03484_amd as P
    P.load()
    return P


def _sim(tpm, w, rcrit, rrem=None, **opts):
    s = tpm.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, **opts)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, rcrit)
    if rrem is not None:
        s.set_removal_radii(rrem)
    s.set_particles(w.r, w.v)
    return s


def _workload(n, seed, permute=False):
    w = W.giants_100k(n=n, seed=seed)
    if permute:
        p = np.array([2, 0, 3, 1])
        w.mu, w.rp, w.vp, w.rcrit = w.mu[p], w.rp[p], w.vp[p], w.rcrit[p]
    return w


def _ephemeris(orc, w, T, rp, dt=None):
    """The oracle's planet table and velocities in the caller's planet order:
    the oracle's planet map takes the planets sorted by semi-major axis (its
    Jacobi order, as the library sorts them), so they are sorted for it and
    the columns put back in the caller's order."""
    rn = np.linalg.norm(rp, axis=1)
    a = 1.0 / (2.0 / rn - np.sum(w.vp ** 2, axis=1) / (w.mu0 + w.mu))
    order = np.argsort(a, kind="stable")
    e = orc.ephemeris(w.mu0, w.mu[order], rp[order], w.vp[order], T, w.dt if dt is None else dt,
                      keep_velocities=True)
    table, vtable = e.table.copy(), e.vtable.copy()
    for k, c in enumerate(order):
        table[:, 3 * c:3 * c + 3] = e.table[:, 3 * k:3 * k + 3]
        vtable[:, 3 * c:3 * c + 3] = e.vtable[:, 3 * k:3 * k + 3]
    return table, vtable


def _handoff_reference(orc, w, T, rrem, M, universal, idx=None, dt=None):
    """Oracle result of the hand-off run on the oracle's own planet table, and
    each particle's near-threshold flag and spread.  A particle is
    near-threshold when its removal record changes as the hand-off, removal
    or escape radius moves by 1e-9 relative, or under one of the conditioning
    probes (a one-ulp change of its start or of the first planet's, the
    contracted build): such a removal is decided at the level of rounding.
    idx: the particles to run (all by default)."""
    sel = slice(None) if idx is None else idx
    r0, v0 = w.r[sel], w.v[sel]
    dt = w.dt if dt is None else dt

    def run(table, vtable, rr=r0, f=1.0):
        return orc.particles_handoff(w.mu0, w.mu, w.rcrit * f, rrem * f, w.rmax * f, table,
                                     vtable, dt, rr, v0, T, substeps=M,
                                     kepler_iters=w.kepler_iters, universal=universal)

    table, vtable = _ephemeris(orc, w, T, w.rp, dt)
    res = run(table, vtable)
    near = np.zeros(len(r0), bool)
    for f in (1 - 1e-9, 1 + 1e-9):
        alt = run(table, vtable, f=f)
        near |= (alt.deact_step != res.deact_step) | (alt.reason != res.reason)

    def response(pert):
        flip = (pert.deact_step != res.deact_step) | (pert.reason != res.reason)
        sp = np.maximum(np.linalg.norm(pert.r - res.r, axis=1) / np.linalg.norm(res.r, axis=1),
                        np.linalg.norm(pert.v - res.v, axis=1) / np.linalg.norm(res.v, axis=1))
        sp[flip] = np.inf
        return sp, flip

    sp1, f1 = response(run(table, vtable, rr=r0 * (1 + np.finfo(float).eps)))
    rp1 = w.rp.copy()
    rp1[0, 0] *= 1 + np.finfo(float).eps
    sp2, f2 = response(run(*_ephemeris(orc, w, T, rp1, dt)))
    with orc.rounding_probe():
        sp3, f3 = response(run(*_ephemeris(orc, w, T, w.rp, dt)))
    near |= f1 | f2 | f3
    return res, near, np.maximum(np.maximum(sp1, sp2), sp3), table


@pytest.mark.parametrize("universal", [False, True])
def test_one_substep_equals_plain_map(tpm, universal):
    """handoff_substeps = 1: the hand-off run (hand-off radius 0.5 au, removal
    radius 0.05 au) equals the plain run with 0.05 au as its encounter radius,
    bit for bit, over chunks of 256 steps (the ring slots, and so the
    encounter stream's ordering, are reused many times); hand-offs happen."""
    w = _workload(4096, 81)
    T = 3000
    rrem = np.full(w.np_, 0.05)
    print(f"[one-substep] n={w.n} T={T} universal={universal}", flush=True)
    s = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=1, chunk_steps=256,
             universal_drift=universal)
    s.integrate(T, w.dt)
    got, st = s.particles(), s.stats()
    ref = _sim(tpm, w, rrem, chunk_steps=256, universal_drift=universal)
    ref.integrate(T, w.dt)
    want = ref.particles()
    print(f"handoffs {st['handoffs']} removed {np.sum(want['reason'] != 0)}", flush=True)
    assert st["handoffs"] > 100
    for k in KEYS:
        assert np.array_equal(got[k], want[k]), k
    assert st["n_active"] == np.sum(want["reason"] == tpm.ACTIVE)
    assert np.array_equal(s.planets()[0], ref.planets()[0])


@pytest.mark.parametrize("M,universal,permute,kiters", [(16, True, False, 5), (4, False, True, 5),
                                                         (8, True, False, 8)])
def test_handoff_matches_oracle(tpm, orc, M, universal, permute, kiters):
    """M substeps per encounter step against the oracle (hand-off radius
    0.5 au, removal radii 0.03..0.06 au per planet, given in caller order;
    planets permuted in one case; a Newton count other than the method's five,
    which runs the kernels that read it at run time, in one): identical
    removal records outside the near-threshold set, states within the parity
    bar, and as many hand-offs as the oracle has particles that reached the
    hand-off radius."""
    w = _workload(4096, 82, permute)
    w.kepler_iters = kiters
    T = 3000
    rrem = np.array([0.03, 0.04, 0.05, 0.06])
    print(f"[oracle M={M} universal={universal} permute={permute} k={kiters}] n={w.n} T={T}",
          flush=True)
    s = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=M, chunk_steps=512,
             universal_drift=universal)
    s.integrate(T, w.dt)
    got, st = s.particles(), s.stats()
    res, near, spread, table = _handoff_reference(orc, w, T, rrem, M, universal)
    # reached the hand-off radius: took an encounter step, was removed within
    # a removal radius, or ends the run within the hand-off radius (handed off
    # at the last step boundary, with no step left to take)
    last = table[T, :3 * w.np_].reshape(w.np_, 3)
    at_end = (res.reason == orc.ACTIVE) & np.any(
        np.linalg.norm(res.r[:, None, :] - last[None], axis=2) < w.rcrit[None], axis=1)
    reached = (res.encounter_steps > 0) | (res.reason == orc.ENCOUNTER) | at_end
    print(f"handoffs {st['handoffs']} oracle reached {reached.sum()} encounter steps "
          f"{res.encounter_steps.sum()} near {near.sum()}; reasons GPU "
          f"{np.bincount(got['reason'], minlength=4)} oracle {np.bincount(res.reason, minlength=4)}",
          flush=True)
    err = np.maximum(np.linalg.norm(got["r"] - res.r, axis=1) / np.linalg.norm(res.r, axis=1),
                     np.linalg.norm(got["v"] - res.v, axis=1) / np.linalg.norm(res.v, axis=1))
    for i in np.argsort(-err)[:5]:
        print(f"  particle {i}: err {err[i]:.3e} spread {spread[i]:.3e} encounter steps "
              f"{res.encounter_steps[i]} removal GPU {got['deact_step'][i]}/{got['reason'][i]} "
              f"oracle {res.deact_step[i]}/{res.reason[i]}", flush=True)
    assert reached.sum() > 100
    _compare(got, res, near, spread, f"handoff M={M}")
    assert abs(st["handoffs"] - reached.sum()) <= near.sum(), (st["handoffs"], reached.sum())


def test_handoff_backwards_matches_oracle(tpm, orc):
    """The hand-off integrating backwards in time (dt < 0: the interpolants'
    velocity terms change sign with the step) against the oracle, to the
    parity bar."""
    w = _workload(4096, 87)
    T = 2500
    rrem = np.full(w.np_, 0.05)
    print(f"[backwards] n={w.n} T={T}", flush=True)
    s = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, universal_drift=True, chunk_steps=700)
    s.integrate(T, -w.dt)
    got, st = s.particles(), s.stats()
    res, near, spread, _ = _handoff_reference(orc, w, T, rrem, 8, True, dt=-w.dt)
    print(f"handoffs {st['handoffs']} encounter steps {res.encounter_steps.sum()}", flush=True)
    assert st["handoffs"] > 100
    _compare(got, res, near, spread, "handoff backwards")


def test_handoff_without_planets_or_particles(tpm):
    """No planets: nothing is handed off and the run equals the plain one bit
    for bit; no particles: the call runs and leaves nothing behind."""
    w = _workload(512, 88)
    empty = np.zeros(0)
    a = tpm.Simulation(r_escape=w.rmax, handoff_substeps=8)
    b = tpm.Simulation(r_escape=w.rmax)
    for s in (a, b):
        s.set_central(w.mu0)
        s.set_planets(empty, np.zeros((0, 3)), np.zeros((0, 3)), empty)
        s.set_particles(w.r, w.v)
    a.set_removal_radii(empty)
    a.integrate(1500, w.dt)
    b.integrate(1500, w.dt)
    pa, pb = a.particles(), b.particles()
    assert a.stats()["handoffs"] == 0
    for k in KEYS:
        assert np.array_equal(pa[k], pb[k]), k
    c = _sim(tpm, w, w.rcrit, np.full(w.np_, 0.05), handoff_substeps=8)
    c.set_particles(np.zeros((0, 3)), np.zeros((0, 3)))
    c.integrate(100, w.dt)
    assert c.stats()["handoffs"] == 0 and c.stats()["step"] == 100


def test_handoff_split_calls_are_bitwise(tpm):
    """One call of 3000 steps and three calls of 700, 1100 and 1200 give the
    same particles and planets bit for bit: survivors of the encounter list
    rejoin the working set at each call's end and, still within the hand-off
    radius, are handed off again at the next call's first step."""
    w = _workload(4096, 83)
    rrem = np.full(w.np_, 0.05)
    print(f"[split] n={w.n}", flush=True)
    a = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=384)
    a.integrate(3000, w.dt)
    b = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=384)
    for k in (700, 1100, 1200):
        b.integrate(k, w.dt)
    pa, pb = a.particles(), b.particles()
    print(f"handoffs {a.stats()['handoffs']} / last call {b.stats()['handoffs']}", flush=True)
    assert a.stats()["handoffs"] > 100
    for k in KEYS:
        assert np.array_equal(pa[k], pb[k]), k
    assert np.array_equal(a.planets()[0], b.planets()[0])
    assert a.stats()["step"] == b.stats()["step"] == 3000


def test_handoff_continues_from_a_state_blob(tpm):
    """A hand-off run continued in a new simulation from tpm_get_state /
    tpm_set_state (removal radii set again, as set_state clears them) equals
    the uninterrupted run bit for bit."""
    w = _workload(2048, 90)
    rrem = np.full(w.np_, 0.05)
    print(f"[state] n={w.n}", flush=True)
    a = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=512)
    a.integrate(2600, w.dt)
    b = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=512)
    b.integrate(1100, w.dt)
    blob = b.get_state()
    b.close()
    c = tpm.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, handoff_substeps=8,
                       chunk_steps=512)
    c.set_state(blob)
    with pytest.raises(tpm.TpmError) as e:
        c.integrate(10, w.dt)                       # the removal radii went with set_state
    assert e.value.code == tpm.TPM_ESTATE
    c.set_removal_radii(rrem)
    c.integrate(1500, w.dt)
    pa, pc = a.particles(), c.particles()
    assert a.stats()["handoffs"] > 20
    for k in KEYS:
        assert np.array_equal(pa[k], pc[k]), k
    assert np.array_equal(a.planets()[0], c.planets()[0])
    assert c.stats()["step"] == 2600


def test_handoff_long_call_runs_in_pieces(tpm, monkeypatch):
    """A call whose planet rows exceed the hand-off ring's budget (set low
    through TPM_HANDOFF_RING_BYTES: 18 chunks of 256 steps) runs as several
    calls: the same particles, planets and step count, bit for bit, as with
    the default budget, and the statistics add up over the pieces."""
    w = _workload(2048, 89)
    rrem = np.full(w.np_, 0.05)
    T = 10_000
    print(f"[pieces] n={w.n} T={T}", flush=True)
    a = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=256)
    a.integrate(T, w.dt)
    monkeypatch.setenv("TPM_HANDOFF_RING_BYTES", str(1 << 20))
    b = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, chunk_steps=256)
    b.integrate(T, w.dt)
    pa, pb = a.particles(), b.particles()
    sa, sb = a.stats(), b.stats()
    print(f"handoffs {sa['handoffs']} / in pieces {sb['handoffs']}, chunks {sa['chunks']} / "
          f"{sb['chunks']}", flush=True)
    for k in KEYS:
        assert np.array_equal(pa[k], pb[k]), k
    assert np.array_equal(a.planets()[0], b.planets()[0])
    assert sb["step"] == T and sb["handoffs"] >= sa["handoffs"] > 50
    assert sb["active_particle_steps"] == sa["active_particle_steps"]


def test_handoff_does_not_depend_on_tuning(tpm):
    """The hand-off run is the same bit for bit under other work-queue shapes,
    chunk lengths and compaction intervals (the chunks decide when the
    encounter list is advanced, the list's lanes nothing else), with the
    eccentricity-binned order and with the universal drift."""
    w = _workload(4096, 86)
    rrem = np.full(w.np_, 0.05)
    print(f"[tuning] n={w.n}", flush=True)
    base = None
    for opts in ({}, {"chunk_steps": 200, "resync_chunks": 3, "sub_chunks": 4, "waves_per_simd": 2},
                 {"chunk_steps": 1000, "block_threads": 256, "sub_chunks": 16, "sort_by_e": True}):
        s = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=8, universal_drift=True, **opts)
        s.integrate(2500, w.dt)
        p = s.particles()
        if base is None:
            base = p
            assert s.stats()["handoffs"] > 100
            continue
        for k in KEYS:
            assert np.array_equal(p[k], base[k]), (opts, k)


def test_handoff_full_size_sampled(tpm, orc):
    """At the 100,000-particle giant-planet shape with the default chunking,
    16 substeps: every particle the GPU removed within a removal radius plus
    1,500 random others, run by the oracle one by one on its own planet
    table, match to the parity bar."""
    w = _workload(100_000, 84)
    T = 2000
    rrem = np.full(w.np_, 0.05)
    print(f"[full-size] n={w.n} T={T}", flush=True)
    s = _sim(tpm, w, w.rcrit, rrem, handoff_substeps=16, universal_drift=True)
    s.integrate(T, w.dt)
    got, st = s.particles(), s.stats()
    rng = np.random.default_rng(5)
    idx = np.union1d(np.flatnonzero(got["reason"] == tpm.ENCOUNTER),
                     rng.choice(w.n, 1500, replace=False))
    res, near, spread, _ = _handoff_reference(orc, w, T, rrem, 16, True, idx=idx)
    print(f"handoffs {st['handoffs']} sampled {idx.size} removed-by-encounter "
          f"{np.sum(got['reason'] == tpm.ENCOUNTER)}", flush=True)
    assert np.sum(got["reason"] == tpm.ENCOUNTER) > 100
    _compare({k: got[k][idx] for k in KEYS}, res, near, spread, "handoff full size")


def test_handoff_refusals(tpm, monkeypatch):
    """The hand-off needs removal radii and the on-device planet map, and does
    not run with the diagnostics, the derivatives, the many-system call or the
    no-allocation call; bad options and radii are refused."""
    import ctypes as C

    from paper_2011_03484_amd import _lib
    w = _workload(256, 85)
    with pytest.raises(tpm.TpmError) as e:
        tpm.Simulation(handoff_substeps=5000)
    assert e.value.code == tpm.TPM_EINVAL
    s = tpm.Simulation(handoff_substeps=4)
    with pytest.raises(tpm.TpmError) as e:
        s.set_removal_radii([])
    assert e.value.code == tpm.TPM_ESTATE
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    s.set_particles(w.r, w.v)
    with pytest.raises(tpm.TpmError) as e:
        s.integrate(10, w.dt)                       # no removal radii yet
    assert e.value.code == tpm.TPM_ESTATE
    for bad in ([0.05, 0.05, 0.0, 0.05], [0.05, np.inf, 0.05, 0.05], [0.05, -1, 0.05, 0.05]):
        with pytest.raises(tpm.TpmError) as e:
            s.set_removal_radii(bad)
        assert e.value.code == tpm.TPM_EINVAL
    s.set_removal_radii(np.full(4, 0.05))
    s.set_diagnostics(10)
    with pytest.raises(tpm.TpmError) as e:
        s.integrate(10, w.dt)
    assert e.value.code == tpm.TPM_ESTATE
    s.close()
    s = _sim(tpm, w, w.rcrit, np.full(4, 0.05), handoff_substeps=4)
    s.set_planet_table(s.planet_table(20, w.dt))
    with pytest.raises(tpm.TpmError) as e:
        s.integrate(10, w.dt)
    assert e.value.code == tpm.TPM_ESTATE
    # a new planet set clears the removal radii
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    with pytest.raises(tpm.TpmError) as e:
        s.integrate(10, w.dt)
    assert e.value.code == tpm.TPM_ESTATE
    rc = _lib.load().tpm_ad_forward(s._h, 0, None, None, 10, C.c_double(w.dt), 5, None, None,
                                    None, None, None)
    assert rc == tpm.TPM_ESTATE
    s.close()
    real = _lib.default_options

    def with_handoff():
        o = real()
        o.handoff_substeps = 4
        return o
    monkeypatch.setattr(_lib, "default_options", with_handoff)
    with pytest.raises(tpm.TpmError) as e:
        tpm.batch_integrate([w], nsteps=10)
    assert e.value.code == tpm.TPM_EINVAL
    with pytest.raises(tpm.TpmError) as e:
        tpm.integrate_static(w.mu0, w.mu, w.rp, w.vp, w.rcrit, 0, 0, 10, w.dt, 0, 0, 0, 0, 0,
                             n=0)
    assert e.value.code == tpm.TPM_EINVAL
