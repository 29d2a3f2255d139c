"""tpm_integrate_static (the run that allocates nothing) against the
simulation-object path (tpm_set_* + tpm_integrate + tpm_get_particles) on the
same inputs: bit-identical particle results, through the C ABI, on two calls
in a row, the second with fewer particles and planets (the library's fixed
device array keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2011_03484_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tpm():
    import paper_2011_03484_amd as P
    P.load()
    return P


def _reference(tpm, w, T):
    s = tpm.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    s.set_particles(w.r, w.v)
    try:
        s.integrate(T, w.dt)
    except tpm.PlanetEncounterError:
        pass
    out = s.particles()
    s.close()
    return out


def _static(tpm, w, T, **opts):
    import torch
    dev = torch.device("cuda", 0)
    n = w.n
    d_r = torch.tensor(w.r, dtype=torch.float64, device=dev)
    d_v = torch.tensor(w.v, dtype=torch.float64, device=dev)
    # outputs start as garbage, so that nothing unwritten can pass
    r_out = torch.full((n, 3), np.nan, dtype=torch.float64, device=dev)
    v_out = torch.full((n, 3), np.nan, dtype=torch.float64, device=dev)
    step = torch.full((n,), -7, dtype=torch.int64, device=dev)
    reason = torch.full((n,), -7, dtype=torch.int32, device=dev)
    planet = torch.full((n,), -7, dtype=torch.int32, device=dev)
    info = torch.full((2,), 99, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    tpm.integrate_static(w.mu0, w.mu, w.rp, w.vp, w.rcrit, d_r.data_ptr(), d_v.data_ptr(), T, w.dt,
                         r_out.data_ptr(), v_out.data_ptr(), step.data_ptr(), reason.data_ptr(),
                         planet.data_ptr(), info.data_ptr(), stream, r_escape=w.rmax,
                         kepler_iters=w.kepler_iters, n=n, **opts)
    torch.cuda.synchronize()
    return ({"r": r_out.cpu().numpy(), "v": v_out.cpu().numpy(), "deact_step": step.cpu().numpy(),
             "reason": reason.cpu().numpy(), "planet": planet.cpu().numpy()},
            info.cpu().numpy())


def test_static_run_equals_simulation_path(tpm):
    cases = [(W.giants_100k(n=5000, seed=31), 3000, {"chunk_steps": 1000}),
             (W.single_planet(n=700, seed=32), 2500, {})]
    for w, T, opts in cases:
        ref = _reference(tpm, w, T)
        got, info = _static(tpm, w, T, **opts)
        print(f"[{w.name}] n={w.n} planets={w.np_} removed={np.sum(ref['reason'] != 0)} "
              f"info={info.tolist()}", flush=True)
        assert np.sum(ref["reason"] != 0) > 0
        for k in ("r", "v", "deact_step", "reason", "planet"):
            assert np.array_equal(got[k], ref[k]), (w.name, k)
        assert info.tolist() == [-1, 0]


def test_static_run_refuses_oversized_requests(tpm):
    w = W.single_planet(n=4, seed=33)
    with pytest.raises(tpm.TpmError):
        tpm.integrate_static(w.mu0, w.mu, w.rp, w.vp, w.rcrit, 1, 1, 10, w.dt, 1, 1, 1, 1, 1,
                             n=(1 << 18) + 1)
    with pytest.raises(tpm.TpmError):
        tpm.integrate_static(w.mu0, w.mu, w.rp, w.vp, w.rcrit, 1, 1, 10, w.dt, 1, 1, 1, 1, 1,
                             n=4, chunk_steps=8193)
