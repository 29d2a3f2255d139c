"""Calibration of the GPU parity bar on the CPU (no GPU).

The element-wise parity tests hold a regular particle (one whose oracle
trajectory moves by at most 1e-12 under a one-ulp change of its initial
position, and end to end of the first planet's) to the plain 1e-11, and a
chaotic particle to 100 x that one-ulp spread.  Both rest on how far a change
of the rounding sequence alone moves a trajectory.  This test measures it with
the oracle itself: the same source built a second time with FMA contraction
(every a*b+c fused, a different rounding at almost every step, the kind of
difference the GPU's explicit FMAs make) against the strict-IEEE build, on the
workloads the parity tests use.  No GPU result enters.
"""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W

REGULAR_SPREAD = 1e-12
CHAOS_FACTOR = 100.0
POS_TOL = 1e-11


def _has_fma():
    try:
        return " fma " in " " + open("/proc/cpuinfo").read().replace("\n", " ") + " "
    except OSError:
        return False


@pytest.fixture(scope="module")
def contracted(orc):
    if not _has_fma():
        pytest.skip("host CPU has no FMA instructions")
    return orc.rounding_probe


@pytest.mark.parametrize("name,make,T,limit,max_moved", [
    ("single_planet", lambda: W.single_planet(n=1024), 1000, 25.0, 0),
    ("adjoint_16k", lambda: W.adjoint_16k(n=2000), 1000, 25.0, 0),
    ("giants_100k", lambda: W.giants_100k(n=3000), 1000, 25.0, 0),
    ("single_planet_10k", lambda: W.single_planet(n=512), 10_000, 70.0, 4),
])
def test_chaos_multiplier(orc, contracted, name, make, T, limit, max_moved):
    """End to end (each build's own planet table): regular particles stay
    within 1e-11 of the strict build; chaotic ones within `limit` x spread,
    which leaves the parity bar's factor 100 a margin (measured: at most 12 at
    1,000 steps, 42 at 10,000).  Removal records that a one-ulp change leaves
    in place are identical at 1,000 steps; at 10,000 a few of them move under
    the rounding change (they are chaotic past what a one-ulp probe shows) and
    are counted, not compared."""
    from test_gpu_parity import _oracle_reference
    w = make()
    eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, T, w.dt)
    res, near, spread = _oracle_reference(orc, w, T, eph.table, rounding=False)

    def run():
        tab = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, T, w.dt).table
        return orc.particles(w.mu0, w.mu, w.rcrit, w.rmax, tab, w.dt, w.r, w.v, T,
                             kepler_iters=w.kepler_iters)

    with contracted():
        alt = run()
    stable = ~near & np.isfinite(spread)
    moved = stable & ((alt.deact_step != res.deact_step) | (alt.planet != res.planet))
    cmp_ = stable & ~moved
    err = np.maximum(np.linalg.norm(alt.r - res.r, axis=1) / np.linalg.norm(res.r, axis=1),
                     np.linalg.norm(alt.v - res.v, axis=1) / np.linalg.norm(res.v, axis=1))
    regular = cmp_ & (spread <= REGULAR_SPREAD)
    chaotic = cmp_ & (spread > REGULAR_SPREAD)
    ratio = err[chaotic] / spread[chaotic] if chaotic.any() else np.zeros(1)
    print(f"[{name}] regular {regular.sum()} max err {err[regular].max() if regular.any() else 0:.2e}; "
          f"chaotic {chaotic.sum()} max err/spread {ratio.max():.2f}; removal records moved "
          f"{moved.sum()}", flush=True)
    assert moved.sum() <= max_moved
    assert np.all(err[regular] <= POS_TOL)
    assert ratio.max() <= limit <= CHAOS_FACTOR
