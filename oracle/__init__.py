"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle of the test-particle map.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.cpp`` (plain C++,
``-O2 -ffp-contract=off``, no fast-math, OpenMP over particles) through ctypes
and adds textbook element conversions used by the invariant tests.  It imports
nothing from the HIP package and the HIP package imports nothing from it.

Entry points (each cites the passage of Zhang & Gladman 2021 it follows):

* :func:`ephemeris`  - planets by the Wisdom-Holman map in Jacobi coordinates
  (sec. 2.2, planet integration; Jacobi definitions in sec. 2.2) writing the
  table of heliocentric planet positions and the indirect term h0 (sec. 2.2).
* :func:`particles`  - the test-particle leapfrog: half kick, Kepler drift by
  the difference form of Kepler's equation with f and g functions, half kick,
  and the encounter / escape / Kepler-failure deactivation (sec. 2.2).
* :func:`run`        - both of the above.
* :func:`particles_handoff` - the particle map with the close-encounter
  hand-off (sec. 5): encounter steps taken in substeps with the planets
  interpolated between table rows.
* :func:`history_table` - the planet table interpolated from a history of
  planet states instead of the planet map (sec. 2.2, planet positions from
  any source).
* :func:`tangent`, :func:`stm`, :func:`adjoint` - the exact derivative of the
  discrete particle map by the complex-step method (Squire & Trapp 1998).
* :func:`kepler_solve`, :func:`kepler_fixedk`, :func:`drift` - unit pieces.
* :func:`elements`, :func:`mean_longitudes`, :func:`diagnostics` - osculating
  elements and the sampled diagnostics of the applications: e_max and its
  step (sec. 3.3), resonant angles and the 10-degree libration criterion
  (sec. 4.1, 4.2).
* :func:`count_ops`, :func:`flops_per_step` - the FP64 operation count of one
  particle step of the method (the algorithmic work of the throughput
  roofline), tallied on the oracle's own step.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with every a*b+c contracted into one fused operation:
# a different rounding at almost every step of the same arithmetic.  Not an
# oracle of its own; a probe of how far rounding alone moves a trajectory.
_LIB_FMA = os.path.join(_HERE, "liboracle_fma.so")

ACTIVE, ENCOUNTER, ESCAPE, KEPLER = 0, 1, 2, 3
KEPLER_FTOL = 1e-13

_FLAGS = {_LIB: ["-ffp-contract=off", "-fno-fast-math"],
          _LIB_FMA: ["-ffp-contract=fast", "-mfma", "-fno-fast-math"]}


def _compile(lib: str, force: bool):
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", *_FLAGS[lib], "-fopenmp", "-fPIC", "-shared", _SRC,
               "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with g++ (strict IEEE doubles, OpenMP), and the
    contracted build ``liboracle_fma.so`` (see rounding_probe)."""
    _compile(_LIB, force)
    _compile(_LIB_FMA, force)
    return _LIB


_lib = None
_lib_fma = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            _compile(_LIB, True)
        _lib = _declare(C.CDLL(_LIB))
    return _lib


class rounding_probe:
    """Context manager: inside it, every entry point runs the contracted build
    of the same source (a different rounding sequence of the same method).  How
    far a result moves under it measures how strongly that particle's
    trajectory amplifies per-step rounding, which a one-ulp change of the
    initial state alone can underestimate (near-parabolic passages)."""

    def __enter__(self):
        global _lib, _lib_fma
        if _lib_fma is None:
            if not os.path.exists(_LIB_FMA) or os.path.getmtime(_LIB_FMA) < os.path.getmtime(_SRC):
                _compile(_LIB_FMA, True)
            _lib_fma = _declare(C.CDLL(_LIB_FMA))
        self._saved = _load()
        _lib = _lib_fma
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _declare(lib):
    """Argument and result types of the library's entry points."""
    d, i, i64 = C.c_double, C.c_int, C.c_int64
    P = C.c_void_p
    lib.orc_kepler_solve.argtypes = [d, d, d, C.POINTER(i)]
    lib.orc_kepler_solve.restype = d
    lib.orc_kepler_fixedk.argtypes = [d, d, d, i, C.POINTER(d)]
    lib.orc_kepler_fixedk.restype = d
    lib.orc_drift.argtypes = [d, P, P, d, i, d, P]
    lib.orc_drift.restype = i
    lib.orc_ephemeris.argtypes = [d, i, P, P, P, i64, d, P, P, P, P]
    lib.orc_ephemeris.restype = i64
    lib.orc_particles.argtypes = [d, i, P, P, d, P, i64, d, i64, i, d, i64, P, P, P, P, P, i, i]
    lib.orc_drift_universal.argtypes = [d, P, P, d]
    lib.orc_drift_universal.restype = i
    lib.orc_particles.restype = d
    lib.orc_max_threads.argtypes = [i]
    lib.orc_max_threads.restype = i
    lib.orc_tangent.argtypes = [d, i, P, P, d, P, i64, d, i, d, i64, P, P, P, P, P, P, i]
    lib.orc_tangent.restype = None
    lib.orc_count_ops.argtypes = [d, i, P, P, d, P, d, i, d, i64, P, P, P]
    lib.orc_count_ops.restype = i64
    lib.orc_particles_diag.argtypes = [d, i, P, P, d, P, i64, d, i64, i, d, i64, P, P, P, P, P,
                                       i, i64, P, i, P, P, P, P, P, P, P, P]
    lib.orc_particles_diag.restype = d
    lib.orc_history_table.argtypes = [i, P, i64, P, P, P, d, d, i64, P, P]
    lib.orc_history_table.restype = i64
    lib.orc_elements.argtypes = [d, i64, P, P, P]
    lib.orc_elements.restype = None
    lib.orc_mean_longitudes.argtypes = [d, i64, P, P, P]
    lib.orc_mean_longitudes.restype = None
    lib.orc_particles_handoff.argtypes = [d, i, P, P, P, d, P, P, i64, d, i64, i, d, i, i, i64, P,
                                          P, P, P, P, P, i]
    lib.orc_particles_handoff.restype = d
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


# ----------------------------------------------------------------- unit pieces
def kepler_solve(ec: float, es: float, dM: float) -> tuple[float, int]:
    """Converged root of x - ec sin x + es (1 - cos x) = dM (sec. 2.2)."""
    it = C.c_int(0)
    x = _load().orc_kepler_solve(float(ec), float(es), float(dM), C.byref(it))
    return x, it.value


def kepler_fixedk(ec: float, es: float, dM: float, k: int = 5) -> tuple[float, float]:
    """Fixed-k Newton reference iteration; returns (x_k, F(x_k)) (sec. 2.2)."""
    F = C.c_double(0.0)
    x = _load().orc_kepler_fixedk(float(ec), float(es), float(dM), int(k), C.byref(F))
    return x, F.value


def drift(mu: float, r, v, dt: float, kfix: int = -1, ftol: float = KEPLER_FTOL):
    """Two-body f-g drift; returns (ok, r, v, (f, g, fdot, gdot))."""
    r = _f64(r, (3,)).copy()
    v = _f64(v, (3,)).copy()
    fg = np.zeros(4)
    ok = _load().orc_drift(float(mu), _ptr(r), _ptr(v), float(dt), int(kfix), float(ftol), _ptr(fg))
    return bool(ok), r, v, fg


def drift_universal(mu: float, r, v, dt: float):
    """Universal-variable two-body drift; returns (ok, r, v)."""
    r = _f64(r, (3,)).copy()
    v = _f64(v, (3,)).copy()
    ok = _load().orc_drift_universal(float(mu), _ptr(r), _ptr(v), float(dt))
    return bool(ok), r, v


# ------------------------------------------------------------------- planets
@dataclass
class Ephemeris:
    table: np.ndarray       # (nsteps+1, 3np+3): r_1..r_np, h0 (heliocentric)
    r_final: np.ndarray     # (np, 3)
    v_final: np.ndarray     # (np, 3)
    flag: int               # -1 ok; >= 0 first step with a planet pair inside a mutual Hill radius; -2 drift failure
    vtable: np.ndarray | None = None   # (nsteps+1, 3np) heliocentric planet velocities, if asked for


def ephemeris(mu0: float, mu, rp, vp, nsteps: int, dt: float, keep_table: bool = True,
              keep_velocities: bool = False) -> Ephemeris:
    """Planet table by the Jacobi Wisdom-Holman map (sec. 2.2)."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    rp = _f64(rp, (npl, 3))
    vp = _f64(vp, (npl, 3))
    table = np.zeros((nsteps + 1, 3 * npl + 3)) if keep_table else None
    vtable = np.zeros((nsteps + 1, 3 * npl)) if keep_velocities else None
    rf = np.zeros((npl, 3))
    vf = np.zeros((npl, 3))
    flag = _load().orc_ephemeris(float(mu0), npl, _ptr(mu), _ptr(rp), _ptr(vp), int(nsteps),
                                 float(dt), _ptr(table) if table is not None else None,
                                 _ptr(rf), _ptr(vf), _ptr(vtable) if vtable is not None else None)
    return Ephemeris(table, rf, vf, int(flag), vtable)


def history_table(mu, t, hr, hv, t0: float, dt: float, nsteps: int, keep_velocities=False):
    """Planet table (and optionally velocities) at times t0 + n dt, n = 0..nsteps,
    by cubic Hermite interpolation of a history of planet states: t[nrec],
    hr, hv [nrec][np][3] heliocentric (sec. 2.2: planet positions from any
    source, such as a history file).  Raises if a row lies outside the
    history."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    t = _f64(t).reshape(-1)
    hr, hv = _f64(hr, (t.shape[0], npl, 3)), _f64(hv, (t.shape[0], npl, 3))
    table = np.zeros((nsteps + 1, 3 * npl + 3))
    vt = np.zeros((nsteps + 1, npl, 3)) if keep_velocities else None
    bad = _load().orc_history_table(npl, _ptr(mu), t.shape[0], _ptr(t), _ptr(hr), _ptr(hv),
                                    float(t0), float(dt), int(nsteps), _ptr(table),
                                    _ptr(vt) if vt is not None else None)
    if bad >= 0:
        raise ValueError(f"row {bad} lies outside the planet history")
    return (table, vt.reshape(nsteps + 1, 3 * npl)) if keep_velocities else table


# ------------------------------------------------------------------ particles
@dataclass
class Result:
    r: np.ndarray
    v: np.ndarray
    deact_step: np.ndarray
    reason: np.ndarray
    planet: np.ndarray
    seconds: float = 0.0


def particles(mu0: float, mu, rcrit, rmax: float, table, dt: float, r, v, nsteps: int | None = None,
              step0: int = 0, kepler_iters: int = 5, ftol: float = KEPLER_FTOL,
              nthreads: int = 0, universal: bool = False) -> Result:
    """Particles through the given planet table (sec. 2.2 leapfrog + deactivation);
    with universal, drifts the elliptic solve refuses use universal variables
    instead of removing the particle."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    rcrit = _f64(rcrit).reshape(-1)
    table = _f64(table)
    if nsteps is None:
        nsteps = table.shape[0] - 1
    assert table.shape == (nsteps + 1, 3 * npl + 3) or table.shape[0] >= nsteps + 1
    r = _f64(r).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    n = r.shape[0]
    ds = np.zeros(n, dtype=np.int64)
    rs = np.zeros(n, dtype=np.int32)
    pl = np.zeros(n, dtype=np.int32)
    secs = _load().orc_particles(float(mu0), npl, _ptr(mu), _ptr(rcrit), float(rmax), _ptr(table),
                                 int(nsteps), float(dt), int(step0), int(kepler_iters), float(ftol),
                                 n, _ptr(r), _ptr(v), _ptr(ds), _ptr(rs), _ptr(pl), int(nthreads),
                                 int(bool(universal)))
    return Result(r, v, ds, rs, pl, secs)


@dataclass
class HandoffResult(Result):
    encounter_steps: np.ndarray = None   # encounter steps taken per particle


def particles_handoff(mu0: float, mu, r_enc, r_rem, rmax: float, table, vtable, dt: float, r, v,
                      nsteps: int | None = None, substeps: int = 32, step0: int = 0,
                      kepler_iters: int = 5, ftol: float = KEPLER_FTOL, universal: bool = False,
                      nthreads: int = 0) -> HandoffResult:
    """Particles with the close-encounter hand-off (sec. 5; the reading is in
    oracle.cpp above run_particle_handoff): a particle within r_enc of a
    planet at a step boundary takes its next step as `substeps` substeps with
    the planets interpolated between the rows (vtable: the planets'
    heliocentric velocities per row, as ephemeris(keep_velocities=True) gives
    them); removal within r_rem, beyond rmax, or on a refused drift."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    r_enc, r_rem = _f64(r_enc).reshape(-1), _f64(r_rem).reshape(-1)
    table, vtable = _f64(table), _f64(vtable)
    if nsteps is None:
        nsteps = table.shape[0] - 1
    assert table.shape[0] >= nsteps + 1 and vtable.shape[0] >= nsteps + 1
    r = _f64(r).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    n = r.shape[0]
    ds = np.zeros(n, dtype=np.int64)
    rs = np.zeros(n, dtype=np.int32)
    pl = np.zeros(n, dtype=np.int32)
    es = np.zeros(n, dtype=np.int64)
    secs = _load().orc_particles_handoff(float(mu0), npl, _ptr(mu), _ptr(r_enc), _ptr(r_rem),
                                         float(rmax), _ptr(table), _ptr(vtable), int(nsteps),
                                         float(dt), int(step0), int(kepler_iters), float(ftol),
                                         int(bool(universal)), int(substeps), n, _ptr(r), _ptr(v),
                                         _ptr(ds), _ptr(rs), _ptr(pl), _ptr(es), int(nthreads))
    return HandoffResult(r, v, ds, rs, pl, secs, es)


def run(w, nsteps: int | None = None, nthreads: int = 0):
    """Ephemeris + particles for a workload object (see the package's workloads)."""
    nsteps = w.nsteps if nsteps is None else nsteps
    eph = ephemeris(w.mu0, w.mu, w.rp, w.vp, nsteps, w.dt)
    res = particles(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r, w.v, nsteps,
                    kepler_iters=w.kepler_iters, nthreads=nthreads)
    return eph, res


def max_threads(nthreads: int = 0) -> int:
    return int(_load().orc_max_threads(int(nthreads)))


# ------------------------------------------------------------- derivatives
def tangent(mu0, mu, rcrit, rmax, table, dt, r, v, dr, dv, nsteps=None, kepler_iters=5,
            ftol=KEPLER_FTOL, nthreads=0):
    """Directional derivative of the final (r, v) of each particle along (dr, dv),
    exact to rounding by the complex step."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    rcrit = _f64(rcrit).reshape(-1)
    table = _f64(table)
    if nsteps is None:
        nsteps = table.shape[0] - 1
    r, v, dr, dv = (_f64(x).reshape(-1, 3) for x in (r, v, dr, dv))
    n = r.shape[0]
    dro = np.zeros((n, 3))
    dvo = np.zeros((n, 3))
    _load().orc_tangent(float(mu0), npl, _ptr(mu), _ptr(rcrit), float(rmax), _ptr(table),
                        int(nsteps), float(dt), int(kepler_iters), float(ftol), n, _ptr(r),
                        _ptr(v), _ptr(dr), _ptr(dv), _ptr(dro), _ptr(dvo), int(nthreads))
    return dro, dvo


def stm(mu0, mu, rcrit, rmax, table, dt, r, v, nsteps=None, kepler_iters=5, nthreads=0):
    """6x6 state-transition matrix d(r_T, v_T)/d(r_0, v_0) per particle, (n, 6, 6)."""
    r = _f64(r).reshape(-1, 3)
    n = r.shape[0]
    M = np.zeros((n, 6, 6))
    for c in range(6):
        w = np.zeros((n, 6))
        w[:, c] = 1.0
        dro, dvo = tangent(mu0, mu, rcrit, rmax, table, dt, r, v, w[:, :3], w[:, 3:], nsteps,
                           kepler_iters, nthreads=nthreads)
        M[:, :3, c] = dro
        M[:, 3:, c] = dvo
    return M


def adjoint(mu0, mu, rcrit, rmax, table, dt, r, v, gr, gv, nsteps=None, kepler_iters=5, nthreads=0):
    """Vector-Jacobian product: (dL/dr_0, dL/dv_0) = M^T (dL/dr_T, dL/dv_T)."""
    M = stm(mu0, mu, rcrit, rmax, table, dt, r, v, nsteps, kepler_iters, nthreads)
    lam = np.concatenate([_f64(gr).reshape(-1, 3), _f64(gv).reshape(-1, 3)], axis=1)
    g = np.einsum("nij,ni->nj", M, lam)
    return g[:, :3], g[:, 3:]


# ------------------------------------------------------------- diagnostics
def elements(mu: float, r, v) -> np.ndarray:
    """Osculating heliocentric elements (a, e, inc, node, peri, M) of states
    about mu, (n, 6), by the textbook two-body relations."""
    r, v = _f64(r).reshape(-1, 3), _f64(v).reshape(-1, 3)
    out = np.zeros((r.shape[0], 6))
    _load().orc_elements(float(mu), r.shape[0], _ptr(r), _ptr(v), _ptr(out))
    return out


def mean_longitudes(mu: float, r, v) -> np.ndarray:
    """Mean longitudes node + peri + M of states about mu."""
    r, v = _f64(r).reshape(-1, 3), _f64(v).reshape(-1, 3)
    out = np.zeros(r.shape[0])
    _load().orc_mean_longitudes(float(mu), r.shape[0], _ptr(r), _ptr(v), _ptr(out))
    return out


@dataclass
class Diagnostics:
    result: Result
    emax: np.ndarray        # largest sampled osculating e (-1 if never sampled)
    emax_step: np.ndarray   # first sample step reaching it (-1)
    flags: np.ndarray       # (n, nres): bit 0 phi within 10 deg of 0, bit 1 within 10 deg of 180
    lo: np.ndarray          # (n, nres): range of phi - 180 deg over the samples, radians
    hi: np.ndarray
    margin: np.ndarray      # (n, nres): least distance of |phi| or |phi - 180 deg| from 10 deg


def diagnostics(mu0, mu, rcrit, rmax, eph: Ephemeris, dt, r, v, nsteps, every, ref=None,
                resonances=(), kepler_iters=5, ftol=KEPLER_FTOL, nthreads=0) -> Diagnostics:
    """Particles through eph.table with the sampled diagnostics of the
    applications: e_max and its step (sec. 3.3), and for each resonance (p, q)
    with planet `ref` the resonant angle p lambda - q lambda_ref - (p - q) varpi
    (sec. 4.1) against the 10-degree libration criterion (sec. 4.2).  Samples
    at step boundaries that are multiples of `every`; the planet's elements use
    mu0 + mu_ref and need eph made with keep_velocities."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    rcrit = _f64(rcrit).reshape(-1)
    table = _f64(eph.table)
    r = _f64(r).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    n = r.shape[0]
    nres = len(resonances)
    assert nres <= 2 and every > 0
    lam_rows = None
    if nres:
        j = int(ref)
        lam_rows = mean_longitudes(mu0 + mu[j], table[:nsteps + 1, 3 * j:3 * j + 3],
                                   eph.vtable[:nsteps + 1, 3 * j:3 * j + 3])
    pq = np.array([x for x, _ in resonances] or [0], np.int32)
    qq = np.array([y for _, y in resonances] or [0], np.int32)
    ds = np.zeros(n, np.int64)
    rs = np.zeros(n, np.int32)
    pl = np.zeros(n, np.int32)
    emax = np.zeros(n)
    estep = np.zeros(n, np.int64)
    flags = np.zeros((n, max(nres, 1)), np.int32)
    lo = np.zeros((n, max(nres, 1)))
    hi = np.zeros((n, max(nres, 1)))
    margin = np.zeros((n, max(nres, 1)))
    secs = _load().orc_particles_diag(
        float(mu0), npl, _ptr(mu), _ptr(rcrit), float(rmax), _ptr(table), int(nsteps), float(dt),
        0, int(kepler_iters), float(ftol), n, _ptr(r), _ptr(v), _ptr(ds), _ptr(rs), _ptr(pl),
        int(nthreads), int(every), _ptr(lam_rows) if lam_rows is not None else None, nres,
        _ptr(pq), _ptr(qq), _ptr(emax), _ptr(estep), _ptr(flags), _ptr(lo), _ptr(hi), _ptr(margin))
    return Diagnostics(Result(r, v, ds, rs, pl, secs), emax, estep, flags[:, :nres], lo[:, :nres],
                       hi[:, :nres], margin[:, :nres])


# ------------------------------------------------------- operation count
# FP64 flops per counted operation (the rule of the throughput roofline):
# add, subtract and multiply 1; a reciprocal 9 (a hardware estimate and two
# Newton steps y + y (1 - b y) of two FMAs each); a square root 12 (a
# reciprocal-square-root estimate, two Newton steps of one multiply and two
# FMAs, one multiply by x); a sine-cosine pair 39 (a two-constant reduction by
# pi/2 of one multiply and two FMAs, x^2, two degree-8 polynomials in x^2 by
# Horner's rule, one multiply by x).  FMA = 2 flops.
OP_WEIGHTS = {"add": 1, "mul": 1, "rcp": 9, "sqrt": 12, "sincos": 39}


def count_ops(mu0, mu, rcrit, rmax, table, dt, r, v, kepler_iters=5, ftol=KEPLER_FTOL):
    """Operations of one step of the method's particle map, per particle
    (adds, multiplies, reciprocals, square roots, sine-cosine pairs; rows of -1
    for particles removed within two steps), tallied by running the oracle's
    own particle step on a counting number type.  table needs three rows."""
    mu = _f64(mu).reshape(-1)
    npl = mu.shape[0]
    rcrit = _f64(rcrit).reshape(-1)
    table = _f64(table)
    assert table.shape[0] >= 3 and table.shape[1] == 3 * npl + 3
    r, v = _f64(r).reshape(-1, 3), _f64(v).reshape(-1, 3)
    n = r.shape[0]
    out = np.zeros((n, 5), np.int64)
    _load().orc_count_ops(float(mu0), npl, _ptr(mu), _ptr(rcrit), float(rmax), _ptr(table),
                          float(dt), int(kepler_iters), float(ftol), n, _ptr(r), _ptr(v), _ptr(out))
    return out


def flops_per_step(counts) -> float:
    """Mean FP64 flops of one particle step from count_ops rows (OP_WEIGHTS)."""
    c = np.asarray(counts)
    c = c[c[:, 0] >= 0]
    w = np.array([OP_WEIGHTS[k] for k in ("add", "mul", "rcp", "sqrt", "sincos")])
    return float((c @ w).mean())


# ----------------------------------------------------- textbook element helpers
def cartesian_to_elements(mu, r, v):
    """Heliocentric (r, v) -> (a, e, inc, node, peri, M), textbook relations."""
    r = np.atleast_2d(_f64(r))
    v = np.atleast_2d(_f64(v))
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), r.shape[:1])
    rn = np.linalg.norm(r, axis=1)
    v2 = np.sum(v * v, axis=1)
    h = np.cross(r, v)
    hn = np.linalg.norm(h, axis=1)
    a = 1.0 / (2.0 / rn - v2 / mu)
    evec = np.cross(v, h) / mu[:, None] - r / rn[:, None]
    e = np.linalg.norm(evec, axis=1)
    inc = np.arccos(np.clip(h[:, 2] / hn, -1.0, 1.0))
    node = np.arctan2(h[:, 0], -h[:, 1])
    nvec = np.stack([np.cos(node), np.sin(node), np.zeros_like(node)], axis=1)
    # argument of pericentre, measured in the orbital plane from the node line
    hz = h / hn[:, None]
    mvec = np.cross(hz, nvec)
    peri = np.arctan2(np.sum(evec * mvec, axis=1), np.sum(evec * nvec, axis=1))
    # eccentric anomaly from e cos E = 1 - r/a, e sin E = r.v / sqrt(mu a)
    ecE = 1.0 - rn / a
    esE = np.sum(r * v, axis=1) / np.sqrt(mu * a)
    E = np.arctan2(esE, ecE)
    M = E - esE
    return a, e, inc, node, peri, M


def wrap_angle(x):
    return (np.asarray(x) + math.pi) % (2 * math.pi) - math.pi
