"""GPU tangent and adjoint of the particle map against the oracle.

The oracle's derivatives are the complex-step derivatives of its own map, exact
to rounding; the GPU's are hand-written forward and reverse sweeps.  Besides the
oracle comparison: the dot-product identity <M w, l> = <w, M^T l> between the
GPU's tangent and adjoint, torch.autograd.gradcheck, and central differences
with h = 1e-7 on the loss sum |r_T|^2.
"""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2011_03484_amd as P
    from paper_2011_03484_amd import autograd as AG
    P.load()
    return torch, P, AG


def _sim(P, w):
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    return s


def _t(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(n=256, T=1000, seed=None):
    return W.adjoint_16k(n=n, seed=seed).subset(nsteps=T)


def test_ad_forward_matches_integrate(env):
    torch, P, AG = env
    w = _case(n=512, T=700)
    s = _sim(P, w)
    rT, vT, step, reason = AG.integrate(s, _t(torch, w.r), _t(torch, w.v), w.nsteps, w.dt, 100)
    g = P.run_workload(w)
    assert np.array_equal(step.cpu().numpy(), g["deact_step"])
    assert np.array_equal(reason.cpu().numpy(), g["reason"])
    err = np.abs(rT.cpu().numpy() - g["r"]).max() / np.abs(g["r"]).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("k", [5, 8])
def test_tangent_and_adjoint_match_oracle(env, orc, k):
    """Tangent and adjoint against the oracle's complex-step state-transition
    matrices, with the default five Newton steps and with eight (the general
    count of the derivative kernels)."""
    torch, P, AG = env
    w = _case(n=128, T=600)
    w.kepler_iters = k
    s = _sim(P, w)
    rT, vT, step, reason = AG.integrate(s, _t(torch, w.r), _t(torch, w.v), w.nsteps, w.dt, 100)
    eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, w.nsteps, w.dt)
    ref = orc.particles(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r, w.v, w.nsteps,
                        kepler_iters=k)
    same = ref.deact_step == step.cpu().numpy()
    M = orc.stm(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r, w.v, w.nsteps, kepler_iters=k)
    rng = np.random.default_rng(3)
    dr, dv = rng.normal(size=(w.n, 3)), rng.normal(size=(w.n, 3))
    tr, tv = AG.tangent(s, _t(torch, dr), _t(torch, dv))
    tan = np.concatenate([tr.cpu().numpy(), tv.cpu().numpy()], 1)
    tan_ref = np.einsum("nij,nj->ni", M, np.concatenate([dr, dv], 1))
    gr, gv = rng.normal(size=(w.n, 3)), rng.normal(size=(w.n, 3))
    r0 = _t(torch, w.r).requires_grad_(True)
    v0 = _t(torch, w.v).requires_grad_(True)
    rT, vT, _, _ = AG.integrate(s, r0, v0, w.nsteps, w.dt, 100)
    (rT * _t(torch, gr)).sum().add((vT * _t(torch, gv)).sum()).backward()
    adj = np.concatenate([r0.grad.cpu().numpy(), v0.grad.cpu().numpy()], 1)
    adj_ref = np.einsum("nij,ni->nj", M, np.concatenate([gr, gv], 1))
    norm = np.linalg.norm(M, axis=(1, 2))
    et = np.linalg.norm(tan - tan_ref, axis=1) / (np.linalg.norm(tan_ref, axis=1) + 1e-300)
    ea = np.linalg.norm(adj - adj_ref, axis=1) / (np.linalg.norm(adj_ref, axis=1) + 1e-300)
    ok = same & (norm < 1e4)
    print(f"tangent max rel err {et[ok].max():.2e}, adjoint {ea[ok].max():.2e}, "
          f"|M| median {np.median(norm):.1f}, compared {ok.sum()}/{w.n}", flush=True)
    assert ok.sum() > 0.5 * w.n
    assert et[ok].max() < 1e-8 and ea[ok].max() < 1e-8


def test_dot_product_identity(env):
    torch, P, AG = env
    w = _case(n=2048, T=1500)
    s = _sim(P, w)
    r0 = _t(torch, w.r).requires_grad_(True)
    v0 = _t(torch, w.v).requires_grad_(True)
    rT, vT, step, _ = AG.integrate(s, r0, v0, w.nsteps, w.dt, 250)
    rng = np.random.default_rng(5)
    dr, dv, gr, gv = (_t(torch, rng.normal(size=(w.n, 3))) for _ in range(4))
    (rT * gr).sum().add((vT * gv).sum()).backward()
    tr, tv = AG.tangent(s, dr, dv)
    lhs = ((tr * gr).sum(1) + (tv * gv).sum(1)).cpu().numpy()
    rhs = ((dr * r0.grad).sum(1) + (dv * v0.grad).sum(1)).cpu().numpy()
    # <J d, g> = <d, J^T g> per particle.  Rounding in either side is bounded
    # relative to |J d||g| and |d||J^T g| (Cauchy-Schwarz), not to the dot
    # products themselves, which may cancel.  Each of the T steps of a sweep
    # rounds about 300 FP64 operations once each, relative to those norms, and
    # the errors add up at most linearly: 300 T u, u = 2^-53 (5e-11 at
    # T = 1,500).
    nrm = lambda a, b: torch.sqrt((a * a).sum(1) + (b * b).sum(1)).cpu().numpy()
    scale = nrm(tr, tv) * nrm(gr, gv) + nrm(dr, dv) * nrm(r0.grad, v0.grad) + 1e-300
    rel = np.abs(lhs - rhs) / scale
    rel_dot = np.abs(lhs - rhs) / (np.abs(lhs) + np.abs(rhs) + 1e-300)
    print(f"dot-product identity: max rel (norm-scaled) {rel.max():.2e}, "
          f"(dot-scaled) {rel_dot.max():.2e}", flush=True)
    assert rel.max() < 300 * w.nsteps * (np.finfo(float).eps / 2)


def test_gradcheck_small(env):
    torch, P, AG = env
    w = _case(n=4, T=40)
    s = _sim(P, w)
    r0 = _t(torch, w.r).requires_grad_(True)
    v0 = _t(torch, w.v).requires_grad_(True)

    def f(r, v):
        rT, vT, _, _ = AG.integrate(s, r, v, w.nsteps, w.dt, 16)
        return rT, vT

    assert torch.autograd.gradcheck(f, (r0, v0), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_gradient_vs_central_differences(env):
    """Loss sum |r_T|^2, per-particle central differences with h = 1e-7 (all
    particles perturbed at once, one component per run); particles whose
    Jacobian norm stays below 1e3 and whose removal step does not move."""
    torch, P, AG = env
    w = _case(n=1024, T=2000)
    s = _sim(P, w)
    r0 = _t(torch, w.r).requires_grad_(True)
    v0 = _t(torch, w.v).requires_grad_(True)
    rT, vT, step, _ = AG.integrate(s, r0, v0, w.nsteps, w.dt, 200)
    (rT ** 2).sum().backward()
    grad = np.concatenate([r0.grad.cpu().numpy(), v0.grad.cpu().numpy()], 1)
    base_step = step.cpu().numpy()
    h = 1e-7
    X = np.concatenate([w.r, w.v], 1)
    fd = np.zeros_like(X)
    stable = np.ones(w.n, bool)
    with torch.no_grad():
        for c in range(6):
            vals = []
            for sign in (1, -1):
                Xp = X.copy()
                Xp[:, c] += sign * h
                rp, vp, sp, _ = AG.integrate(s, _t(torch, Xp[:, :3]), _t(torch, Xp[:, 3:]),
                                             w.nsteps, w.dt, 200)
                vals.append((rp ** 2).sum(1).cpu().numpy())
                stable &= sp.cpu().numpy() == base_step
            fd[:, c] = (vals[0] - vals[1]) / (2 * h)
    # Jacobian-norm screen from the tangent along each axis
    rT, vT, _, _ = AG.integrate(s, _t(torch, w.r), _t(torch, w.v), w.nsteps, w.dt, 200)
    norm = np.zeros(w.n)
    for c in range(6):
        e = np.zeros((w.n, 6))
        e[:, c] = 1
        tr, tv = AG.tangent(s, _t(torch, e[:, :3]), _t(torch, e[:, 3:]))
        norm = np.maximum(norm, np.linalg.norm(torch.cat([tr, tv], 1).cpu().numpy(), axis=1))
    ok = stable & (norm < 1e3)
    rel = np.linalg.norm(fd - grad, axis=1) / np.linalg.norm(grad, axis=1)
    frac = np.mean(rel[ok] < 1e-6)
    print(f"FD check: {ok.sum()}/{w.n} well-conditioned, {frac:.3f} within 1e-6, "
          f"median rel {np.median(rel[ok]):.2e}", flush=True)
    assert ok.sum() > 0.3 * w.n
    assert frac > 0.95


def test_full_size_derivatives_sampled(env, orc):
    """The 16,384-particle derivative workload (checkpoint every 1,000 steps),
    2,000 steps: tangent and adjoint of every 128th particle against the
    oracle's complex-step state-transition matrix."""
    torch, P, AG = env
    w = W.adjoint_16k().subset(nsteps=2000)
    s = _sim(P, w)
    r0 = _t(torch, w.r).requires_grad_(True)
    v0 = _t(torch, w.v).requires_grad_(True)
    rT, vT, step, _ = AG.integrate(s, r0, v0, w.nsteps, w.dt, 1000)
    rng = np.random.default_rng(11)
    dr, dv = rng.normal(size=(w.n, 3)), rng.normal(size=(w.n, 3))
    tr, tv = AG.tangent(s, _t(torch, dr), _t(torch, dv))
    gr, gv = rng.normal(size=(w.n, 3)), rng.normal(size=(w.n, 3))
    (rT * _t(torch, gr)).sum().add((vT * _t(torch, gv)).sum()).backward()
    idx = np.arange(0, w.n, 128)
    eph = orc.ephemeris(w.mu0, w.mu, w.rp, w.vp, w.nsteps, w.dt)
    ref = orc.particles(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r[idx], w.v[idx], w.nsteps)
    M = orc.stm(w.mu0, w.mu, w.rcrit, w.rmax, eph.table, w.dt, w.r[idx], w.v[idx], w.nsteps)
    same = ref.deact_step == step.cpu().numpy()[idx]
    tan = np.concatenate([tr.cpu().numpy()[idx], tv.cpu().numpy()[idx]], 1)
    tan_ref = np.einsum("nij,nj->ni", M, np.concatenate([dr[idx], dv[idx]], 1))
    adj = np.concatenate([r0.grad.cpu().numpy()[idx], v0.grad.cpu().numpy()[idx]], 1)
    adj_ref = np.einsum("nij,ni->nj", M, np.concatenate([gr[idx], gv[idx]], 1))
    norm = np.linalg.norm(M, axis=(1, 2))
    et = np.linalg.norm(tan - tan_ref, axis=1) / (np.linalg.norm(tan_ref, axis=1) + 1e-300)
    ea = np.linalg.norm(adj - adj_ref, axis=1) / (np.linalg.norm(adj_ref, axis=1) + 1e-300)
    ok = same & (norm < 1e4)
    print(f"full-size derivatives: tangent {et[ok].max():.2e}, adjoint {ea[ok].max():.2e}, "
          f"compared {ok.sum()}/{len(idx)}", flush=True)
    assert ok.sum() > 0.5 * len(idx)
    assert et[ok].max() < 1e-8 and ea[ok].max() < 1e-8
