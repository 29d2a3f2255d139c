"""torch.autograd binding of the library's tangent and adjoint (argument marshalling only).

``TPMVSFunction.apply(r0, v0, sim, nsteps, dt, ckpt_every)`` integrates the
particles (float64 CUDA tensors of shape (n, 3), heliocentric) through the
planets set on ``sim`` and returns ``(rT, vT, deact_step, reason)``.  Its
backward is the library's adjoint: the run is cut into segments of
``ckpt_every`` steps whose starting states are kept; each segment is recomputed
from its checkpoint and swept backwards (tpm_ad_backward).  The planets are not
differentiated.  All work is enqueued on torch's current stream.

A simulation holds the checkpoints of its last forward only; a backward whose
forward is no longer the latest one first re-runs that forward (same inputs,
same result) to rebuild them.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib


def _bind():
    return _lib.load()


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float64):
        raise TypeError("expected a float64 CUDA tensor")
    return t.contiguous()


def _p(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class TPMVSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r0, v0, sim, nsteps: int, dt: float, ckpt_every: int = 1000):
        lib = _bind()
        r0, v0 = _dev(r0), _dev(v0)
        n = r0.shape[0]
        rT, vT = torch.empty_like(r0), torch.empty_like(v0)
        step = torch.empty(n, dtype=torch.int64, device=r0.device)
        reason = torch.empty(n, dtype=torch.int32, device=r0.device)
        _lib._check(lib.tpm_ad_forward(sim._h, n, _p(r0), _p(v0), int(nsteps), float(dt),
                                       int(ckpt_every), _p(rT), _p(vT), _p(step), _p(reason),
                                       _stream()))
        sim._ad_generation = getattr(sim, "_ad_generation", 0) + 1
        ctx.sim = sim
        ctx.generation = sim._ad_generation
        ctx.args = (n, int(nsteps), float(dt), int(ckpt_every))
        ctx.save_for_backward(r0, v0)
        ctx.mark_non_differentiable(step, reason)
        return rT, vT, step, reason

    @staticmethod
    def backward(ctx, gRT, gVT, _gstep, _greason):
        sim = ctx.sim
        lib = _bind()
        n, nsteps, dt, ckpt = ctx.args
        r0, v0 = ctx.saved_tensors
        if sim._ad_generation != ctx.generation:
            # another forward replaced the checkpoints: rebuild this one's
            scratch = [torch.empty_like(r0), torch.empty_like(v0)]
            _lib._check(lib.tpm_ad_forward(sim._h, n, _p(r0), _p(v0), nsteps, dt, ckpt,
                                           _p(scratch[0]), _p(scratch[1]), None, None,
                                           _stream()))
            sim._ad_generation += 1
            ctx.generation = sim._ad_generation
        dev = r0.device
        gRT = torch.zeros(n, 3, dtype=torch.float64, device=dev) if gRT is None else _dev(gRT)
        gVT = torch.zeros(n, 3, dtype=torch.float64, device=dev) if gVT is None else _dev(gVT)
        gR0, gV0 = torch.empty_like(gRT), torch.empty_like(gVT)
        _lib._check(lib.tpm_ad_backward(sim._h, _p(gRT), _p(gVT), _p(gR0), _p(gV0), _stream()))
        return gR0, gV0, None, None, None, None


def integrate(sim, r0, v0, nsteps: int, dt: float, ckpt_every: int = 1000):
    """Differentiable integration; returns (rT, vT, deact_step, reason)."""
    return TPMVSFunction.apply(r0, v0, sim, nsteps, dt, ckpt_every)


def tangent(sim, dR0, dV0):
    """Directional derivative of the last forward's final state along (dR0, dV0)."""
    lib = _bind()
    dR0, dV0 = _dev(dR0), _dev(dV0)
    dRT, dVT = torch.empty_like(dR0), torch.empty_like(dV0)
    _lib._check(lib.tpm_ad_tangent(sim._h, _p(dR0), _p(dV0), _p(dRT), _p(dVT), _stream()))
    return dRT, dVT
