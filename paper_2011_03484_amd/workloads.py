"""Seeded synthetic inputs for the test-particle integrator.

This module only draws initial conditions.  It holds none of the integrator's
arithmetic: it converts drawn osculating elements to Cartesian states with the
textbook two-body relations, sorts planets by semi-major axis (the Jacobi order
of sec. 2.2) and builds encounter radii from the Hill radius
R_H = a_p (m_p / (3 m_0))^(1/3) of sec. 2.2.  Both the HIP path and the oracle are
fed from here; nothing in it calls either of them.

Units: au, yr, solar masses; mu = G m with G m_sun = 4 pi^2 au^3 / yr^2.

Workloads (sizes as in the performance study of sec. 2.3 and the applications of
secs. 3-4, synthetic stand-ins for their real planet initial conditions):

  * ``single_planet``  - Sun + one circular planet (m = 9.55e-4, a = 5.2),
    1,024 particles a ~ U[6, 10], e ~ U[0, 0.1], i ~ U[0, 5 deg]; dt = 0.5 yr,
    10,000 steps; deactivation at 3 R_H or r > 100 au.
  * ``giants_100k``    - Sun + four giant planets (masses 9.55e-4, 2.86e-4,
    4.37e-5, 5.15e-5; a = 5.20, 9.55, 19.2, 30.1; e ~ U[0, 0.05], i ~ U[0, 2 deg],
    random phases), 100,000 particles a ~ U[20, 29], e ~ U[0, 0.05),
    i ~ U[0, 1 deg); dt = 120 d, 1e6 steps; 0.5 au from any planet, r > 1000 au.
  * ``resonant_200k``  - same planets, 200,000 particles a ~ U[54, 64],
    e ~ U[0.1, 0.5], i ~ U[0, 20 deg]; dt = 120 d, 1e7 steps; 1 R_H, r > 1000 au.
  * ``adjoint_16k``    - same planets, 16,384 particles of the single-planet
    distribution; dt = 120 d, 1e5 steps; 3 R_H, r > 100 au.
  * ``batched_512``    - 512 independent systems (see :func:`make_batched`).
  * ``high_e``         - same planets, particles over the applications' a range
    (a ~ U[20, 70]) at high eccentricity: 85% e ~ U[0.5, 0.99], 10% near-parabolic
    e ~ U[0.99, 0.9999], 5% made unbound (velocity scaled to v^2 = 2.4 mu0/r);
    dt = 120 d; 1 R_H, r > 1000 au.  The case the Kepler-solver paragraph of
    sec. 2.2 sets aside (e >= 0.8 and unbound orbits).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MU_SUN = 4.0 * math.pi ** 2          # au^3 / yr^2
DAY = 1.0 / 365.25                    # yr
SEED_BASE = 2011034840

GIANT_MASSES = (9.55e-4, 2.86e-4, 4.37e-5, 5.15e-5)
GIANT_A = (5.20, 9.55, 19.2, 30.1)


@dataclass
class Workload:
    """One system: central mass, planets, particles and run parameters."""
    name: str
    mu0: float
    mu: np.ndarray          # (np,)
    rp: np.ndarray          # (np, 3) heliocentric positions
    vp: np.ndarray          # (np, 3) heliocentric velocities
    rcrit: np.ndarray       # (np,) encounter radius per planet
    rmax: float             # escape radius (<= 0 disables)
    r: np.ndarray           # (n, 3) particle heliocentric positions
    v: np.ndarray           # (n, 3)
    dt: float
    nsteps: int
    kepler_iters: int = 5
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    @property
    def np_(self) -> int:
        return int(self.mu.shape[0])

    def subset(self, n: int | None = None, nsteps: int | None = None) -> "Workload":
        """The same system with the first ``n`` particles and ``nsteps`` steps."""
        n = self.n if n is None else min(n, self.n)
        return Workload(self.name, self.mu0, self.mu.copy(), self.rp.copy(), self.vp.copy(),
                        self.rcrit.copy(), self.rmax, self.r[:n].copy(), self.v[:n].copy(),
                        self.dt, self.nsteps if nsteps is None else int(nsteps),
                        self.kepler_iters, dict(self.meta))


def solve_kepler_mean(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly E from mean anomaly M (E - e sin E = M), vectorised."""
    M = np.asarray(M, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    E = M + e * np.sin(M)
    for _ in range(60):
        dE = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - dE
        if np.all(np.abs(dE) < 1e-15):
            break
    return E


def elements_to_cartesian(mu, a, e, inc, node, peri, M):
    """Textbook elliptic elements -> heliocentric (r, v); all angles in radians.

    Returns arrays of shape (n, 3).
    """
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), np.shape(a))
    a, e, inc, node, peri, M = (np.asarray(x, dtype=np.float64) for x in (a, e, inc, node, peri, M))
    E = solve_kepler_mean(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    # perifocal frame
    xp = a * (cE - e)
    yp = a * b * sE
    rr = a * (1.0 - e * cE)
    nmean = np.sqrt(mu / a ** 3)
    vxp = -a * nmean * sE * a / rr
    vyp = a * nmean * b * cE * a / rr
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si], axis=-1)
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si], axis=-1)
    r = xp[..., None] * P + yp[..., None] * Q
    v = vxp[..., None] * P + vyp[..., None] * Q
    return r, v


def hill_radius(mu0: float, mu_p, a_p):
    """Hill radius a_p (m_p / (3 m_0))^(1/3) (sec. 2.2, close-encounter criterion)."""
    return np.asarray(a_p) * np.cbrt(np.asarray(mu_p) / (3.0 * mu0))


def _rng(index: int, seed: int | None):
    return np.random.Generator(np.random.PCG64(SEED_BASE + index if seed is None else seed))


def _giant_planets(rng):
    k = len(GIANT_A)
    a = np.array(GIANT_A)
    e = rng.uniform(0.0, 0.05, k)
    inc = np.deg2rad(rng.uniform(0.0, 2.0, k))
    node, peri, M = (rng.uniform(0.0, 2 * math.pi, k) for _ in range(3))
    mu = MU_SUN * np.array(GIANT_MASSES)
    rp, vp = elements_to_cartesian(MU_SUN + mu, a, e, inc, node, peri, M)
    return mu, rp, vp, a


def _particles(rng, n, amin, amax, emin, emax, imax_deg):
    a = rng.uniform(amin, amax, n)
    e = rng.uniform(emin, emax, n)
    inc = np.deg2rad(rng.uniform(0.0, imax_deg, n))
    node, peri, M = (rng.uniform(0.0, 2 * math.pi, n) for _ in range(3))
    return elements_to_cartesian(MU_SUN, a, e, inc, node, peri, M)


def single_planet(n: int = 1024, seed: int | None = None) -> Workload:
    rng = _rng(0, seed)
    mu = np.array([MU_SUN * 9.55e-4])
    node, peri, M = (rng.uniform(0.0, 2 * math.pi, 1) for _ in range(3))
    rp, vp = elements_to_cartesian(MU_SUN + mu, np.array([5.2]), np.zeros(1), np.zeros(1),
                                   node, peri, M)
    r, v = _particles(rng, n, 6.0, 10.0, 0.0, 0.1, 5.0)
    rcrit = 3.0 * hill_radius(MU_SUN, mu, np.array([5.2]))
    return Workload("single_planet", MU_SUN, mu, rp, vp, rcrit, 100.0, r, v, 0.5, 10_000)


def giants_100k(n: int = 100_000, seed: int | None = None) -> Workload:
    rng = _rng(1, seed)
    mu, rp, vp, a = _giant_planets(rng)
    r, v = _particles(rng, n, 20.0, 29.0, 0.0, 0.05, 1.0)
    rcrit = np.full(4, 0.5)
    return Workload("giants_100k", MU_SUN, mu, rp, vp, rcrit, 1000.0, r, v, 120.0 * DAY, 1_000_000)


def resonant_200k(n: int = 200_000, seed: int | None = None) -> Workload:
    rng = _rng(2, seed)
    mu, rp, vp, a = _giant_planets(rng)
    r, v = _particles(rng, n, 54.0, 64.0, 0.1, 0.5, 20.0)
    rcrit = 1.0 * hill_radius(MU_SUN, mu, a)
    return Workload("resonant_200k", MU_SUN, mu, rp, vp, rcrit, 1000.0, r, v, 120.0 * DAY,
                    10_000_000)


def adjoint_16k(n: int = 16_384, seed: int | None = None) -> Workload:
    rng = _rng(3, seed)
    mu, rp, vp, a = _giant_planets(rng)
    r, v = _particles(rng, n, 6.0, 10.0, 0.0, 0.1, 5.0)
    rcrit = 3.0 * hill_radius(MU_SUN, mu, a)
    return Workload("adjoint_16k", MU_SUN, mu, rp, vp, rcrit, 100.0, r, v, 120.0 * DAY, 100_000,
                    meta={"checkpoint_every": 1000})


def make_batched(nsys: int = 512, seed: int | None = None, nmin: int = 64, nmax: int = 8192,
                 nsteps: int = 100_000) -> list[Workload]:
    """Independent systems: Np ~ U{1..8}; planet masses log-uniform in
    [1e-5, 1e-3] M_sun, a log-uniform in [1, 40] au (at least 6 mutual Hill radii
    apart, by rejection), e < 0.05, i < 2 deg; particles per system log-uniform in
    [nmin, nmax], e < 0.05, i < 1 deg, with a uniform in a gap between two
    planets chosen uniformly (3 R_H clear of each), or in [a_1 + 3 R_H, 2 a_1]
    when Np = 1; dt = 1/30 of the innermost planet's period; 3 R_H, r > 100 au.
    """
    rng = _rng(4, seed)
    systems = []
    for s in range(nsys):
        k = int(rng.integers(1, 9))
        while True:
            m = np.exp(rng.uniform(math.log(1e-5), math.log(1e-3), k))
            a = np.exp(rng.uniform(math.log(1.0), math.log(40.0), k))
            order = np.argsort(a)
            m, a = m[order], a[order]
            ok = True
            for j in range(k - 1):
                rmh = np.cbrt((m[j] + m[j + 1]) / 3.0) * 0.5 * (a[j] + a[j + 1])
                if a[j + 1] - a[j] < 6.0 * rmh:
                    ok = False
                    break
            if ok:
                break
        mu = MU_SUN * m
        e = rng.uniform(0.0, 0.05, k)
        inc = np.deg2rad(rng.uniform(0.0, 2.0, k))
        node, peri, M = (rng.uniform(0.0, 2 * math.pi, k) for _ in range(3))
        rp, vp = elements_to_cartesian(MU_SUN + mu, a, e, inc, node, peri, M)
        rh = hill_radius(MU_SUN, mu, a)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        if k == 1:
            lo, hi = a[0] + 3 * rh[0], 2 * a[0]
        else:
            g = int(rng.integers(0, k - 1))
            lo, hi = a[g] + 3 * rh[g], a[g + 1] - 3 * rh[g + 1]
        r, v = _particles(rng, n, lo, hi, 0.0, 0.05, 1.0)
        period = 2 * math.pi * math.sqrt(a[0] ** 3 / (MU_SUN + mu[0]))
        systems.append(Workload(f"batched_{s}", MU_SUN, mu, rp, vp, 3.0 * rh, 100.0, r, v,
                                period / 30.0, nsteps))
    return systems


def high_e(n: int = 4096, seed: int | None = None) -> Workload:
    rng = _rng(5, seed)
    mu, rp, vp, a = _giant_planets(rng)
    n_np = n // 10
    n_hyp = n // 20
    n_ell = n - n_np - n_hyp
    r1, v1 = _particles(rng, n_ell, 20.0, 70.0, 0.5, 0.99, 20.0)
    r2, v2 = _particles(rng, n_np + n_hyp, 20.0, 70.0, 0.99, 0.9999, 20.0)
    r, v = np.concatenate([r1, r2]), np.concatenate([v1, v2])
    # the last n_hyp: speed raised to v^2 = 2.4 mu0 / r (unbound)
    h = slice(n - n_hyp, n)
    rn = np.linalg.norm(r[h], axis=1)
    v2n = np.sum(v[h] * v[h], axis=1)
    v[h] *= np.sqrt(2.4 * MU_SUN / (rn * v2n))[:, None]
    perm = rng.permutation(n)
    rcrit = 1.0 * hill_radius(MU_SUN, mu, a)
    return Workload("high_e", MU_SUN, mu, rp, vp, rcrit, 1000.0, r[perm], v[perm], 120.0 * DAY,
                    10_000)


WORKLOADS = {
    "single_planet": single_planet,
    "giants_100k": giants_100k,
    "resonant_200k": resonant_200k,
    "adjoint_16k": adjoint_16k,
    "high_e": high_e,
}
