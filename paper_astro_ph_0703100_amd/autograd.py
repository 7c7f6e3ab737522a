"""Differentiable force evaluation and leapfrog rollout (torch.autograd front end).

* ``ForceFn``: forward = ``nbody_force_f64`` (accelerations and potentials from FP64
  positions), backward = ``nbody_force_vjp_f64`` (the hand-written adjoint kernel).
* ``RolloutFn``: forward = ``nbody_leapfrog`` with per-step position checkpoints,
  backward = ``nbody_leapfrog_adjoint`` (reverse KDK with one adjoint kernel call
  per checkpoint).  Gradients flow to the initial positions, velocities and masses.

All arithmetic runs in the library; these classes only allocate tensors, convert
the mass argument to the FP32 the kernels read, and pass pointers and the stream.
Positions and velocities are ``[3, n]`` float64 device tensors, masses ``[n]``
(float32 or float64; gradients come back in the dtype given).
"""
from __future__ import annotations

import torch

from . import _lib
from .api import _check_pos, make_opts, stream_ptr

__all__ = ["ForceFn", "RolloutFn", "force", "rollout"]


def _mass32(mass: torch.Tensor, n: int) -> torch.Tensor:
    if not mass.is_cuda or mass.shape != (n,):
        raise ValueError("mass must be a CUDA tensor of shape [%d]" % n)
    return mass.detach().to(torch.float32).contiguous()


class ForceFn(torch.autograd.Function):
    """(acc [3, n], pot [n]) = F(pos64 [3, n], mass [n]); differentiable in pos and mass."""

    @staticmethod
    def forward(ctx, pos64, mass, eps, precision="comp", centre="system"):
        n = _check_pos(pos64, torch.float64, "pos64")
        m32 = _mass32(mass, n)
        acc = torch.empty((3, n), dtype=torch.float64, device=pos64.device)
        pot = torch.empty(n, dtype=torch.float64, device=pos64.device)
        opts = make_opts(precision=precision, centre=centre)
        _lib.nbody_force_f64(n, pos64.data_ptr(), m32.data_ptr(), float(eps), acc.data_ptr(),
                             pot.data_ptr(), opts, stream_ptr())
        ctx.save_for_backward(pos64, m32)
        ctx.eps, ctx.precision, ctx.centre, ctx.mass_dtype = eps, precision, centre, mass.dtype
        return acc, pot

    @staticmethod
    def backward(ctx, g_acc, g_pot):
        pos64, m32 = ctx.saved_tensors
        n = pos64.shape[1]
        dev = pos64.device
        ga = (g_acc if g_acc is not None else torch.zeros((3, n), dtype=torch.float64, device=dev))
        ga = ga.to(torch.float64).contiguous()
        gp = g_pot.to(torch.float64).contiguous() if g_pot is not None else None
        grad_pos = torch.empty((3, n), dtype=torch.float64, device=dev)
        grad_mass = (torch.empty(n, dtype=torch.float64, device=dev)
                     if ctx.needs_input_grad[1] else None)
        opts = make_opts(precision=ctx.precision, centre=ctx.centre)
        _lib.nbody_force_vjp_f64(n, pos64.data_ptr(), m32.data_ptr(), float(ctx.eps),
                                 ga.data_ptr(), gp.data_ptr() if gp is not None else None,
                                 grad_pos.data_ptr(),
                                 grad_mass.data_ptr() if grad_mass is not None else None,
                                 opts, stream_ptr())
        if grad_mass is not None:
            grad_mass = grad_mass.to(ctx.mass_dtype)
        return (grad_pos if ctx.needs_input_grad[0] else None), grad_mass, None, None, None


class RolloutFn(torch.autograd.Function):
    """(x_T, v_T) after ``nsteps`` KDK steps from (x0, v0); differentiable in x0, v0, mass."""

    @staticmethod
    def forward(ctx, x0, v0, mass, eps, dt, nsteps, precision="comp", centre="system"):
        n = _check_pos(x0, torch.float64, "x0")
        _check_pos(v0, torch.float64, "v0")
        m32 = _mass32(mass, n)
        x = x0.detach().clone()
        v = v0.detach().clone()
        acc = torch.empty((3, n), dtype=torch.float64, device=x0.device)
        traj = torch.empty((nsteps + 1, 3, n), dtype=torch.float64, device=x0.device)
        opts = make_opts(precision=precision, centre=centre)
        _lib.nbody_leapfrog(n, x.data_ptr(), v.data_ptr(), m32.data_ptr(), float(eps), float(dt),
                            int(nsteps), acc.data_ptr(), None, traj.data_ptr(),
                            _lib.NBODY_LF_INIT_ACC, opts, stream_ptr())
        ctx.save_for_backward(traj, m32)
        ctx.eps, ctx.dt, ctx.nsteps = eps, dt, nsteps
        ctx.precision, ctx.centre, ctx.mass_dtype = precision, centre, mass.dtype
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        traj, m32 = ctx.saved_tensors
        n = traj.shape[2]
        dev = traj.device
        xbar = (gx.to(torch.float64).clone() if gx is not None
                else torch.zeros((3, n), dtype=torch.float64, device=dev)).contiguous()
        vbar = (gv.to(torch.float64).clone() if gv is not None
                else torch.zeros((3, n), dtype=torch.float64, device=dev)).contiguous()
        mbar = torch.zeros(n, dtype=torch.float64, device=dev) if ctx.needs_input_grad[2] else None
        opts = make_opts(precision=ctx.precision, centre=ctx.centre)
        _lib.nbody_leapfrog_adjoint(n, traj.data_ptr(), m32.data_ptr(), float(ctx.eps),
                                    float(ctx.dt), int(ctx.nsteps), xbar.data_ptr(),
                                    vbar.data_ptr(), mbar.data_ptr() if mbar is not None else None,
                                    opts, stream_ptr())
        if mbar is not None:
            mbar = mbar.to(ctx.mass_dtype)
        return xbar, vbar, mbar, None, None, None, None, None


def force(pos64, mass, eps, precision="comp", centre="system"):
    return ForceFn.apply(pos64, mass, eps, precision, centre)


def rollout(x0, v0, mass, eps, dt, nsteps, precision="comp", centre="system"):
    return RolloutFn.apply(x0, v0, mass, eps, dt, nsteps, precision, centre)
