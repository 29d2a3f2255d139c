"""ctypes binding of ``libtpmvs.so`` (argument marshalling only).

Every computation happens in the library's HIP kernels; this module converts
numpy arrays to pointers and error codes to exceptions.  The library is loaded
from the package directory; if it is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpmvs.so")

TPM_OK, TPM_EINVAL, TPM_ENOMEM, TPM_EDEVICE, TPM_ESTATE, TPM_EPLANET = 0, -1, -2, -3, -4, -5
ACTIVE, ENCOUNTER, ESCAPE, KEPLER = 0, 1, 2, 3
ERROR_NAMES = {TPM_EINVAL: "EINVAL", TPM_ENOMEM: "ENOMEM", TPM_EDEVICE: "EDEVICE",
               TPM_ESTATE: "ESTATE", TPM_EPLANET: "EPLANET"}


class TpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tpm error {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class PlanetEncounterError(TpmError):
    """Planets came within a mutual Hill radius (results are still valid to read)."""


class Options(C.Structure):
    _fields_ = [("kepler_iters", C.c_int32), ("chunk_steps", C.c_int32),
                ("resync_chunks", C.c_int32), ("block_threads", C.c_int32),
                ("sub_chunks", C.c_int32), ("waves_per_simd", C.c_int32),
                ("r_escape", C.c_double), ("kepler_ftol", C.c_double), ("device", C.c_int32),
                ("time_kernels", C.c_int32), ("universal_drift", C.c_int32),
                ("sort_by_e", C.c_int32), ("handoff_substeps", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_particles", C.c_int64), ("n_active", C.c_int64),
                ("active_particle_steps", C.c_int64), ("wall_ms", C.c_double),
                ("particle_ms", C.c_double), ("ephemeris_ms", C.c_double), ("chunks", C.c_int64),
                ("particle_kernel_ms", C.c_double), ("compactions", C.c_int64),
                ("count_by_reason", C.c_int64 * 4), ("sub_chunks", C.c_int32),
                ("waves_per_simd", C.c_int32), ("block_threads", C.c_int32),
                ("chunk_steps", C.c_int32), ("resync_chunks", C.c_int32),
                ("handoffs", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "count_by_reason"}
        d["count_by_reason"] = list(self.count_by_reason)
        return d


SNAPSHOT_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_void_p, C.c_void_p)


class DiagOptions(C.Structure):
    _fields_ = [("every", C.c_int64), ("ref_planet", C.c_int32), ("nres", C.c_int32),
                ("p", C.c_int32 * 2), ("q", C.c_int32 * 2), ("snapshot", SNAPSHOT_FN),
                ("user", C.c_void_p)]


# Exported symbols and their signatures; the tests check the library against this list
# and include/tpmvs.h.
_P = C.c_void_p
SIGNATURES = {
    "tpm_default_options": (None, [_P]),
    "tpm_create": (C.c_int, [_P, _P]),
    "tpm_destroy": (None, [_P]),
    "tpm_set_central": (C.c_int, [_P, C.c_double]),
    "tpm_set_planets": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "tpm_set_particles": (C.c_int, [_P, C.c_int64, _P, _P]),
    "tpm_set_removal_radii": (C.c_int, [_P, _P]),
    "tpm_integrate": (C.c_int, [_P, C.c_int64, C.c_double]),
    "tpm_get_particles": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "tpm_get_planets": (C.c_int, [_P, _P, _P]),
    "tpm_get_stats": (C.c_int, [_P, _P]),
    "tpm_hill_radius": (C.c_double, [C.c_double, C.c_double, C.c_double]),
    "tpm_last_error": (C.c_char_p, []),
    "tpm_planet_table": (C.c_int, [_P, C.c_int64, C.c_double, _P]),
    "tpm_set_planet_table": (C.c_int, [_P, _P, C.c_int64]),
    "tpm_debug_sincos": (C.c_int, [C.c_int64, _P, _P, _P]),
    "tpm_debug_rsqrt": (C.c_int, [C.c_int64, _P, _P]),
    "tpm_debug_drift": (C.c_int, [C.c_double, C.c_int64, _P, _P, _P, C.c_double, C.c_int32,
                                  C.c_double]),
    "tpm_debug_drift_universal": (C.c_int, [C.c_double, C.c_int64, _P, _P, _P, C.c_double,
                                            C.c_int32]),
    "tpm_ad_forward": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int64, C.c_double, C.c_int32, _P, _P,
                                 _P, _P, _P]),
    "tpm_ad_backward": (C.c_int, [_P] * 6),
    "tpm_ad_tangent": (C.c_int, [_P] * 6),
    "tpm_batch_integrate": (C.c_int, [C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_int64,
                                      _P, _P, _P, _P, _P, _P, _P, _P]),
    "tpm_get_state": (C.c_int, [_P, _P, _P]),
    "tpm_set_diagnostics": (C.c_int, [_P, _P]),
    "tpm_set_planet_history": (C.c_int, [_P, C.c_int64, _P, _P, _P, C.c_double]),
    "tpm_get_diagnostics": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "tpm_set_state": (C.c_int, [_P, _P, C.c_int64]),
    "tpm_integrate_static": (C.c_int, [_P, C.c_double, C.c_int32, _P, _P, _P, _P, C.c_int64, _P, _P,
                                       C.c_int64, C.c_double, _P, _P, _P, _P, _P, _P, _P]),
}

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2011_03484_amd.build` (no CPU fallback exists)")
        # torch bundles a HIP runtime with the same soname as the system one the
        # library links; loading torch first makes both use that one copy (a
        # second copy loaded after the library's leaves the library without a
        # device)
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != TPM_OK:
        msg = load().tpm_last_error().decode()
        if rc == TPM_EPLANET:
            raise PlanetEncounterError(rc, msg)
        raise TpmError(rc, msg)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(shape)
    return a


def default_options() -> Options:
    o = Options()
    load().tpm_default_options(C.byref(o))
    return o


def hill_radius(mu0: float, mu_p: float, a_p: float) -> float:
    return load().tpm_hill_radius(float(mu0), float(mu_p), float(a_p))


class Simulation:
    """One integrator instance on one GPU (see include/tpmvs.h)."""

    def __init__(self, kepler_iters: int = 5, chunk_steps: int = 0, resync_chunks: int = 0,
                 block_threads: int = 0, r_escape: float = 0.0, kepler_ftol: float = 0.0,
                 device: int = 0, time_kernels: bool = False, sub_chunks: int = 0,
                 waves_per_simd: int = 0, universal_drift: bool = False,
                 sort_by_e: bool = False, handoff_substeps: int = 0):
        lib = load()
        o = default_options()
        o.kepler_iters, o.chunk_steps, o.resync_chunks = kepler_iters, chunk_steps, resync_chunks
        o.block_threads, o.r_escape, o.kepler_ftol, o.device = (block_threads, r_escape,
                                                                kepler_ftol, device)
        o.time_kernels = int(bool(time_kernels))
        o.sub_chunks, o.waves_per_simd = sub_chunks, waves_per_simd
        o.universal_drift, o.sort_by_e = int(bool(universal_drift)), int(bool(sort_by_e))
        o.handoff_substeps = int(handoff_substeps)
        h = C.c_void_p()
        _check(lib.tpm_create(C.byref(o), C.byref(h)))
        self._h = h
        self.np = 0
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            load().tpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_central(self, mu0: float):
        _check(load().tpm_set_central(self._h, float(mu0)))

    def set_planets(self, mu, r, v, r_crit):
        mu = _f64(mu, (-1,))
        npl = mu.shape[0]
        r, v = _f64(r, (npl, 3)), _f64(v, (npl, 3))
        rc = _f64(r_crit, (npl,))
        _check(load().tpm_set_planets(self._h, npl, _p(mu), _p(r), _p(v), _p(rc)))
        self.np = npl

    def set_removal_radii(self, r_rem):
        """Per-planet removal radii of the close-encounter hand-off
        (tpm_set_removal_radii; after set_planets)."""
        rr = _f64(r_rem, (self.np,))
        _check(load().tpm_set_removal_radii(self._h, _p(rr)))

    def set_particles(self, r, v):
        r = _f64(r, (-1, 3))
        v = _f64(v, (r.shape[0], 3))
        _check(load().tpm_set_particles(self._h, r.shape[0], _p(r), _p(v)))
        self.n = r.shape[0]

    def integrate(self, nsteps: int, dt: float):
        _check(load().tpm_integrate(self._h, int(nsteps), float(dt)))

    def particles(self):
        n = self.n
        r, v = np.zeros((n, 3)), np.zeros((n, 3))
        st = np.zeros(n, np.int64)
        rs = np.zeros(n, np.int32)
        pl = np.zeros(n, np.int32)
        _check(load().tpm_get_particles(self._h, _p(r), _p(v), _p(st), _p(rs), _p(pl)))
        return {"r": r, "v": v, "deact_step": st, "reason": rs, "planet": pl}

    def planets(self):
        r, v = np.zeros((self.np, 3)), np.zeros((self.np, 3))
        _check(load().tpm_get_planets(self._h, _p(r), _p(v)))
        return r, v

    def stats(self) -> dict:
        s = Stats()
        _check(load().tpm_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def get_state(self) -> bytes:
        """The simulation's whole state as an opaque blob (tpm_get_state)."""
        size = C.c_int64(0)
        _check(load().tpm_get_state(self._h, None, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        _check(load().tpm_get_state(self._h, buf, C.byref(size)))
        return buf.raw[:size.value]

    def set_state(self, blob: bytes):
        """Replace central mass, planets, particles and step count by a blob of
        get_state (tpm_set_state); integrating then continues that run."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(load().tpm_set_state(self._h, buf, len(blob)))
        hdr = np.frombuffer(bytes(blob[:32]), dtype=np.int64)
        self.np = int(np.frombuffer(bytes(blob[12:16]), dtype=np.int32)[0])
        self.n = int(hdr[2])

    def set_diagnostics(self, every: int, ref_planet: int = -1, resonances=(), snapshot=None):
        """Sampled diagnostics every `every` steps (tpm_set_diagnostics):
        e_max and its step, and for each resonance (p, q) with planet
        `ref_planet` the 10-degree flags and the range of phi - 180 degrees.
        `snapshot(step, dict)` (optional) receives copies of r, v, deact_step,
        reason and elements at every sample."""
        o = DiagOptions()
        o.every, o.ref_planet, o.nres = int(every), int(ref_planet), len(resonances)
        for k, (p, q) in enumerate(resonances):
            o.p[k], o.q[k] = int(p), int(q)
        self._snap_cb = None
        if snapshot is not None:
            def cb(user, step, n, r, v, st, rs, el):
                def arr(ptr, dtype, shape):
                    count = int(np.prod(shape))
                    buf = (C.c_char * (count * np.dtype(dtype).itemsize)).from_address(ptr)
                    return np.frombuffer(buf, dtype=dtype).reshape(shape).copy()
                snapshot(int(step), {"r": arr(r, np.float64, (n, 3)), "v": arr(v, np.float64, (n, 3)),
                                     "deact_step": arr(st, np.int64, (n,)),
                                     "reason": arr(rs, np.int32, (n,)),
                                     "elements": arr(el, np.float64, (n, 6))})
            self._snap_cb = SNAPSHOT_FN(cb)
            o.snapshot = self._snap_cb
        self._nres = len(resonances)
        _check(load().tpm_set_diagnostics(self._h, C.byref(o)))

    def diagnostics(self):
        n, k = self.n, max(self._nres, 0)
        emax = np.zeros(n)
        estep = np.zeros(n, np.int64)
        flags = np.zeros((n, k), np.int32)
        lo, hi = np.zeros((n, k)), np.zeros((n, k))
        _check(load().tpm_get_diagnostics(self._h, _p(emax), _p(estep), _p(flags), _p(lo), _p(hi)))
        return {"emax": emax, "emax_step": estep, "flags": flags, "lo": lo, "hi": hi}

    def planet_table(self, nsteps: int, dt: float):
        t = np.zeros((nsteps + 1, 3 * self.np + 3))
        _check(load().tpm_planet_table(self._h, int(nsteps), float(dt), _p(t)))
        return t

    def set_planet_history(self, t, r, v, t0: float = 0.0):
        """Planets from a history of states (tpm_set_planet_history): times
        t[nrec], heliocentric r, v [nrec][np][3]; row n at time t0 + n dt.
        t None turns it off."""
        if t is None:
            _check(load().tpm_set_planet_history(self._h, 0, None, None, None, 0.0))
            return
        t = _f64(t, (-1,))
        r, v = _f64(r, (t.shape[0], self.np, 3)), _f64(v, (t.shape[0], self.np, 3))
        _check(load().tpm_set_planet_history(self._h, t.shape[0], _p(t), _p(r), _p(v), float(t0)))

    def set_planet_table(self, table):
        if table is None:
            _check(load().tpm_set_planet_table(self._h, None, 0))
            return
        t = _f64(table, (-1, 3 * self.np + 3))
        _check(load().tpm_set_planet_table(self._h, _p(t), t.shape[0]))


def debug_sincos(x):
    x = _f64(x, (-1,))
    s, c = np.zeros_like(x), np.zeros_like(x)
    _check(load().tpm_debug_sincos(x.shape[0], _p(x), _p(s), _p(c)))
    return s, c


def debug_rsqrt(x):
    """Columns: 1/sqrt(x), sqrt(x), 1/x, x^-1.5, x^-1.5 (first-order factor)."""
    x = _f64(x, (-1,))
    out = np.zeros((x.shape[0], 5))
    _check(load().tpm_debug_rsqrt(x.shape[0], _p(x), _p(out)))
    return out


def debug_drift(mu, r, v, dt, kepler_iters=5, kepler_ftol=0.0):
    r = _f64(r, (-1, 3))
    v = _f64(v, (r.shape[0], 3))
    rv = np.ascontiguousarray(np.concatenate([r, v], axis=1))
    out = np.zeros_like(rv)
    ok = np.zeros(r.shape[0], np.int32)
    _check(load().tpm_debug_drift(float(mu), r.shape[0], _p(rv), _p(out), _p(ok), float(dt),
                                  int(kepler_iters), float(kepler_ftol)))
    return out[:, :3], out[:, 3:], ok.astype(bool)


def debug_drift_universal(mu, r, v, dt, mode=2):
    """Universal-variable drift (mode 2), or the particle kernel's drift with
    the universal fallback (mode 1); returns (r, v, ok)."""
    r = _f64(r, (-1, 3))
    v = _f64(v, (r.shape[0], 3))
    rv = np.ascontiguousarray(np.concatenate([r, v], axis=1))
    out = np.zeros_like(rv)
    ok = np.zeros(r.shape[0], np.int32)
    _check(load().tpm_debug_drift_universal(float(mu), r.shape[0], _p(rv), _p(out), _p(ok),
                                            float(dt), int(mode)))
    return out[:, :3], out[:, 3:], ok.astype(bool)


def batch_integrate(systems, nsteps=None, r_escape=None, kepler_iters=5, chunk_steps=0,
                    sub_chunks=0, waves_per_simd=0, block_threads=0, resync_chunks=0, strict=True):
    """Integrate many independent systems (workload objects) in one launch.

    Returns (per-system list of result dicts, stats dict).  The stats carry
    ``planet_flag`` per system (-1, or the first step of a planet-planet close
    approach, or -2 for an unbound planet); with ``strict`` any flag raises
    PlanetEncounterError (the results are complete either way)."""
    nsys = len(systems)
    mu0 = np.array([w.mu0 for w in systems], dtype=np.float64)
    poff = np.zeros(nsys + 1, np.int32)
    poff[1:] = np.cumsum([w.np_ for w in systems])
    qoff = np.zeros(nsys + 1, np.int64)
    qoff[1:] = np.cumsum([w.n for w in systems])
    cat = lambda xs, shape: np.ascontiguousarray(np.concatenate(xs) if len(xs) else np.zeros(shape))
    mu_p = cat([w.mu for w in systems], (0,))
    rp = cat([w.rp.reshape(-1, 3) for w in systems], (0, 3))
    vp = cat([w.vp.reshape(-1, 3) for w in systems], (0, 3))
    rc = cat([w.rcrit for w in systems], (0,))
    r = cat([w.r for w in systems], (0, 3))
    v = cat([w.v for w in systems], (0, 3))
    dt = np.array([w.dt for w in systems], dtype=np.float64)
    T = systems[0].nsteps if nsteps is None else int(nsteps)
    o = default_options()
    o.kepler_iters, o.chunk_steps, o.sub_chunks = kepler_iters, chunk_steps, sub_chunks
    o.waves_per_simd, o.block_threads = waves_per_simd, block_threads
    o.resync_chunks = resync_chunks
    o.r_escape = systems[0].rmax if r_escape is None else r_escape
    n = int(qoff[-1])
    ro, vo = np.zeros((n, 3)), np.zeros((n, 3))
    st = np.zeros(n, np.int64)
    rs = np.zeros(n, np.int32)
    pl = np.zeros(n, np.int32)
    stats = Stats()
    flags = np.zeros(nsys, np.int64)
    rc_ = load().tpm_batch_integrate(nsys, _p(mu0), _p(poff), _p(mu_p), _p(rp), _p(vp), _p(rc),
                                     _p(qoff), _p(r), _p(v), _p(dt), T, C.byref(o), _p(ro), _p(vo),
                                     _p(st), _p(rs), _p(pl), C.byref(stats), _p(flags))
    out = [{"r": ro[qoff[i]:qoff[i + 1]], "v": vo[qoff[i]:qoff[i + 1]],
            "deact_step": st[qoff[i]:qoff[i + 1]], "reason": rs[qoff[i]:qoff[i + 1]],
            "planet": pl[qoff[i]:qoff[i + 1]]} for i in range(nsys)]
    sd = stats.as_dict()
    sd["planet_flag"] = flags
    if strict or rc_ != TPM_EPLANET:
        _check(rc_)
    return out, sd


def integrate_static(mu0, mu, rp, vp, rcrit, d_r, d_v, nsteps, dt, d_r_out, d_v_out, d_step,
                     d_reason, d_planet, d_info=None, stream=None, r_escape=0.0, kepler_iters=5,
                     chunk_steps=0, resync_chunks=0, block_threads=0, sub_chunks=0,
                     waves_per_simd=0, device=0, n=None):
    """One run without allocation (tpm_integrate_static).  Planets are host
    arrays; d_* are device addresses (ints, e.g. a torch tensor's data_ptr())
    of [n][3] float64 inputs and of the outputs; stream is a HIP stream handle
    (int) or None.  Returns once the work is enqueued."""
    mu = _f64(mu, (-1,))
    npl = mu.shape[0]
    rp, vp, rc = _f64(rp, (npl, 3)), _f64(vp, (npl, 3)), _f64(rcrit, (npl,))
    o = default_options()
    o.kepler_iters, o.chunk_steps, o.resync_chunks = kepler_iters, chunk_steps, resync_chunks
    o.block_threads, o.sub_chunks, o.waves_per_simd = block_threads, sub_chunks, waves_per_simd
    o.r_escape, o.device = r_escape, device
    vp_ = lambda x: None if x is None else C.c_void_p(int(x))
    _check(load().tpm_integrate_static(C.byref(o), float(mu0), npl, _p(mu), _p(rp), _p(vp), _p(rc),
                                       int(n), vp_(d_r), vp_(d_v), int(nsteps), float(dt),
                                       vp_(d_r_out), vp_(d_v_out), vp_(d_step), vp_(d_reason),
                                       vp_(d_planet), vp_(d_info), vp_(stream)))


def run_workload(w, nsteps=None, **opts):
    """Integrate a workload object (see the workloads module) and return results."""
    sim = Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, **opts)
    sim.set_central(w.mu0)
    sim.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    sim.set_particles(w.r, w.v)
    sim.integrate(w.nsteps if nsteps is None else nsteps, w.dt)
    out = sim.particles()
    out["planets"] = sim.planets()
    out["stats"] = sim.stats()
    sim.close()
    return out
