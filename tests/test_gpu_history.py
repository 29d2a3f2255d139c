"""Planet positions from an interpolated history on the GPU against the oracle.

The paper notes that the planet positions shared by the particles could come
from any source, such as interpolation from a history file (sec. 2.2).  The
history here is a coarse record (every 16 steps) of the oracle's own planet
map; both sides interpolate it by cubic Hermite polynomials (each its own
code) and the particles then run through those rows.
"""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W
from test_gpu_parity import _compare, _oracle_reference

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tpm():
    import paper_2011_03484_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _history(orc, w, nrec, every):
    eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, (nrec - 1) * every, w.dt, keep_velocities=True)
    idx = np.arange(nrec) * every
    t = idx * w.dt
    hr = eph.table[idx, :3 * w.np_].reshape(nrec, w.np_, 3)
    hv = eph.vtable[idx].reshape(nrec, w.np_, 3)
    return t, hr, hv


def _sim(tpm, w, **opts):
    s = tpm.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, **opts)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    return s


def test_history_rows_match_oracle(tpm, orc):
    w = W.giants_100k(n=1)
    t, hr, hv = _history(orc, w, 200, 16)
    T = 3000
    t0 = 0.37 * w.dt          # rows fall between records
    ref = orc.history_table(w.mu, t, hr, hv, t0, w.dt, T)
    s = _sim(tpm, w)
    # planets given out of order: the library sorts them and reports in caller order
    perm = np.array([2, 0, 3, 1])
    s2 = tpm.Simulation(r_escape=w.rmax)
    s2.set_central(w.mu0)
    s2.set_planets(w.mu[perm], w.rp[perm], w.vp[perm], w.rcrit[perm])
    s2.set_planet_history(t, hr[:, perm], hv[:, perm], t0)
    s.set_planet_history(t, hr, hv, t0)
    g = s.planet_table(T, w.dt)
    g2 = s2.planet_table(T, w.dt)
    s.close()
    s2.close()
    pos = np.abs(g[:, :12] - ref[:, :12]).max() / np.abs(ref[:, :12]).max()
    h0 = np.abs(g[:, 12:] - ref[:, 12:]).max() / np.abs(ref[:, 12:]).max()
    print(f"rows: max rel position {pos:.2e}, h0 {h0:.2e}", flush=True)
    assert pos < 1e-14 and h0 < 1e-13
    cols = np.concatenate([np.arange(3 * j, 3 * j + 3) for j in perm] + [np.arange(12, 15)])
    assert np.array_equal(g2, g[:, cols])


@pytest.mark.parametrize("direction", ["forward", "backward"])
def test_particles_through_history(tpm, orc, direction):
    w = W.giants_100k(n=4096, seed=91)
    T = 1000
    t, hr, hv = _history(orc, w, 90, 16)
    if direction == "forward":
        dt, t0 = w.dt, 0.25 * w.dt
    else:
        dt, t0 = -w.dt, t[-1] - 0.5 * w.dt
    w.dt = dt
    table = orc.history_table(w.mu, t, hr, hv, t0, dt, T)
    res, near, spread = _oracle_reference(orc, w, T, table, planet_sensitivity=False)
    s = _sim(tpm, w, chunk_steps=300)
    s.set_planet_history(t, hr, hv, t0)
    s.set_particles(w.r, w.v)
    s.integrate(400, dt)
    s.integrate(600, dt)
    g = s.particles()
    rp, vp = s.planets()
    s.close()
    _compare(g, res, near, spread, f"history {direction}")
    # the planets' state at the current step: the interpolant there
    tab, vt = orc.history_table(w.mu, t, hr, hv, t0 + T * dt, dt, 0, keep_velocities=True)
    assert np.allclose(rp.ravel(), tab[0, :12], rtol=0, atol=1e-13 * np.abs(tab).max())
    assert np.allclose(vp.ravel(), vt[0], rtol=0, atol=1e-13 * np.abs(vt).max())


def test_history_range_is_checked(tpm, orc):
    w = W.giants_100k(n=64)
    t, hr, hv = _history(orc, w, 20, 16)
    s = _sim(tpm, w)
    s.set_planet_history(t, hr, hv, 0.0)
    s.set_particles(w.r, w.v)
    last = int(np.floor(t[-1] / w.dt))
    with pytest.raises(tpm.TpmError) as e:
        s.integrate(last + 1, w.dt)
    assert e.value.code == tpm.TPM_EINVAL
    assert s.stats()["step"] == 0
    s.integrate(last, w.dt)           # the whole history is usable
    assert s.stats()["step"] == last
    with pytest.raises(tpm.TpmError):
        s.set_planet_history(t[::-1], hr, hv, 0.0)     # times must increase
    s.close()
