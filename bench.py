"""Throughput benchmark: FP64 particle-steps per second on one MI355X.

One benchmark step is one whole run of the 100,000-particle, four-giant-planet
workload (dt = 120 d, 1e6 steps by default): planet map, particle kernel,
compaction and final gather, with all inputs already resident in HBM (every
step gets its own simulation object, loaded before the timed region).

Prints one JSON line with the throughput (active particle-steps / wall time of
the timed steps), the roofline of the particle kernel (FP64 ALU bound; HIP
events around every particle launch), and the CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Executed FP64 flops of one active particle-step of the particle kernel at
# four planets and five Newton iterations (FMA = 2, ADD/MUL/transcendental
# = 1), counted from the kernel's loop body (see the design notes' roofline
# section, where the counter cross-check is recorded).
FLOPS_PER_PARTICLE_STEP = {4: 629}
FP64_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "particle_queue_giants_100k_traffic.json")


def kernel_source_hash() -> str:
    """Fingerprint of the HIP sources (traffic counters apply to one version)."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2011_03484_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(particle_steps_per_launch: float):
    """HBM bytes per particle launch: the calibrated FETCH_SIZE + WRITE_SIZE
    bytes per active particle-step of the committed counter runs, times this
    run's particle-steps per launch; None unless the counters were taken on the
    current kernel sources."""
    try:
        import json as _j
        d = _j.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d["bytes_per_particle_step"] * particle_steps_per_launch


def cpu_baseline(w, n_sample: int, steps_sample: int):
    import oracle
    sub = w.subset(n=n_sample)
    t0 = time.perf_counter()
    eph = oracle.ephemeris(sub.mu0, sub.mu, sub.rp, sub.vp, steps_sample, sub.dt)
    t1 = time.perf_counter()
    res = oracle.particles(sub.mu0, sub.mu, sub.rcrit, sub.rmax, eph.table, sub.dt, sub.r, sub.v,
                           steps_sample, kepler_iters=sub.kepler_iters)
    t2 = time.perf_counter()
    import numpy as np
    d = res.deact_step
    active = int(np.where(d < 0, steps_sample, d).sum())
    return {"value": active / (t2 - t0), "unit": "particle-steps/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"first {n_sample} particles x {steps_sample} steps of the same workload "
                      f"(planet map {t1 - t0:.2f} s + particles {res.seconds:.2f} s, "
                      f"{active} active particle-steps)"}


def adjoint_ratio(P, W, torch, nsteps: int, n: int, ckpt: int):
    """Forward (with checkpoints) and backward of loss = sum |r_T|^2 on the
    16,384-particle four-planet workload; returns times and their ratio."""
    from paper_2011_03484_amd import autograd as AG
    w = W.adjoint_16k(n=n)
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    r0 = torch.tensor(w.r, dtype=torch.float64, device="cuda").requires_grad_(True)
    v0 = torch.tensor(w.v, dtype=torch.float64, device="cuda").requires_grad_(True)
    # warm-up on a short run
    rT, vT, _, _ = AG.integrate(s, r0, v0, 2 * ckpt, w.dt, ckpt)
    (rT ** 2).sum().backward()
    r0.grad = v0.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rT, vT, step, reason = AG.integrate(s, r0, v0, nsteps, w.dt, ckpt)
    loss = (rT ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    survivors = int((reason == 0).sum().item())
    s.close()
    return {"workload": f"adjoint_16k: {n} particles, 4 planets, {nsteps} steps, checkpoint every "
                        f"{ckpt}, loss = sum |r_T|^2",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "survivors": survivors}


def batched_run(P, W, nsteps: int):
    """512 independent systems (Np 1..8, ~0.86M particles) in one graph launch."""
    systems = W.make_batched(nsteps=nsteps)
    t0 = time.perf_counter()
    res, st = P.batch_integrate(systems, nsteps=nsteps, strict=False)
    t1 = time.perf_counter()
    n = sum(w.n for w in systems)
    return {"workload": f"batched_512: 512 systems, Np U{{1..8}}, {n} particles, dt = P_inner/30, "
                        f"{nsteps} steps, one HIP-graph launch",
            "value": st["active_particle_steps"] / (st["particle_ms"] / 1e3),
            "unit": "particle-steps/s", "graph_ms": st["particle_ms"],
            "call_s_incl_setup_and_tuning": t1 - t0,
            "active_particle_steps": st["active_particle_steps"],
            "systems_with_planet_close_approach": int((st["planet_flag"] != -1).sum()),
            "queue_shape": {"sub_chunks": st["sub_chunks"], "waves_per_simd": st["waves_per_simd"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsteps", type=int, default=1_000_000, help="time steps per run")
    ap.add_argument("--n", type=int, default=100_000, help="particles")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--resync", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-particles", type=int, default=16384)
    ap.add_argument("--cpu-steps", type=int, default=10000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=100_000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=100_000)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device with a plain copy "
                         "kernel (the reference for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(multi-GPU sharding is described in the design notes, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2011_03484_amd as P
    from paper_2011_03484_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.init()
    w = W.giants_100k(n=args.n)
    T = args.nsteps
    sims = []
    for _ in range(args.warmup + args.steps):
        s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, chunk_steps=args.chunk,
                         resync_chunks=args.resync, block_threads=args.block, time_kernels=True)
        s.set_central(w.mu0)
        s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
        s.set_particles(w.r, w.v)
        sims.append(s)
    for i in range(args.warmup):
        sims[i].integrate(T, w.dt)
        print(f"warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        sims[i].integrate(T, w.dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [sims[i].stats() for i in range(args.warmup, args.warmup + args.steps)]
    secs = t1 - t0
    aps = sum(s["active_particle_steps"] for s in stats)
    kern_ms = sum(s["particle_kernel_ms"] for s in stats)
    launches = sum(s["chunks"] for s in stats)
    eph_ms = sum(s["ephemeris_ms"] for s in stats)
    pstream_ms = sum(s["particle_ms"] for s in stats)
    fpps = FLOPS_PER_PARTICLE_STEP.get(w.np_)
    achieved = fpps * aps / (kern_ms / 1e3) / 1e12 if fpps and kern_ms > 0 else None
    line = {
        "metric": "FP64 particle-steps/sec and % FP64 peak, 1 MI355X; adjoint/forward cost ratio",
        "value": aps / secs,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "giants_100k: Sun + 4 giant planets, 100,000 particles a~U[20,29] au, "
                               "dt=120 d, 1e6 steps per run" if (T == 1_000_000 and args.n == 100_000)
                   else f"giants_100k reduced: {args.n} particles, {T} steps per run",
                   "particles": args.n, "planets": w.np_, "time_steps": T, "dt_days": 120.0,
                   "kepler_iters": w.kepler_iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                     "traffic": measured_traffic(aps / max(launches, 1))},
        "kernel": {"name": "particle_queue<4,5>", "launches": launches,
                   "avg_launch_ms": kern_ms / max(launches, 1),
                   "flops_per_particle_step": fpps,
                   "particle_steps_per_s_kernels_only": aps / (kern_ms / 1e3) if kern_ms else None,
                   "particle_stream_ms": pstream_ms, "ephemeris_stream_ms": eph_ms},
        "active_particle_steps": aps,
        "survivors_per_run": [s["count_by_reason"][0] for s in stats],
    }
    for s in sims:
        s.close()
    if args.copy_calibration_mb > 0:
        # a plain device copy of known size, its source evicted from the
        # last-level cache first by writing a larger buffer
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        flush = torch.empty(4 * nbytes // 8, dtype=torch.float64, device="cuda")
        flush.fill_(2.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del flush
        line["copy_calibration_bytes"] = nbytes
    if not args.no_adjoint:
        line["adjoint"] = adjoint_ratio(P, W, torch, args.adjoint_steps, 16_384, 1000)
        print("adjoint done", file=sys.stderr, flush=True)
    if not args.no_batched:
        line["batched"] = batched_run(P, W, args.batched_steps)
        print("batched done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_particles, args.cpu_steps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
