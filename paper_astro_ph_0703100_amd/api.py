"""Torch-tensor front end of the C ABI (argument marshalling only).

Tensors are device tensors in the library's layout: positions ``[3, n]``
(structure of arrays), masses ``[n]``.  Outputs are allocated here with
``torch.empty`` and filled by the library on the current HIP stream; nothing is
computed in torch.
"""
from __future__ import annotations

import torch

from . import _lib

__all__ = ["make_opts", "force", "force_f64", "leapfrog", "LeapfrogGraph", "BatchPlan",
           "morton_order", "soa", "aos", "stream_ptr"]


def make_opts(precision: str = "comp", centre: str = "system", self_pot: bool = False,
              ipl: int = 0, jtile: int = 0, nseg: int = 0, jlanes: int = 0,
              symmetric: int = 0, workspace: torch.Tensor | None = None):
    o = _lib.nbody_opts_default()
    o.precision = _lib.PRECISIONS[precision]
    o.centre = _lib.CENTRES[centre]
    o.self_pot = int(bool(self_pot))
    o.ipl, o.jtile, o.nseg, o.jlanes = int(ipl), int(jtile), int(nseg), int(jlanes)
    o.symmetric = int(symmetric)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def stream_ptr(stream: torch.cuda.Stream | None = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def soa(x_nx3: torch.Tensor, dtype=None) -> torch.Tensor:
    """``(n, 3)`` -> contiguous ``[3, n]`` (layout conversion of an argument)."""
    t = x_nx3.t()
    return t.to(dtype).contiguous() if dtype is not None else t.contiguous()


def aos(x_3xn: torch.Tensor) -> torch.Tensor:
    """``[3, n]`` -> ``(n, 3)`` view-copy."""
    return x_3xn.t().contiguous()


def _check_pos(pos: torch.Tensor, dtype, name="pos"):
    if not pos.is_cuda or pos.dtype != dtype or pos.dim() != 2 or pos.shape[0] != 3 \
            or not pos.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor of shape [3, n]" % (name, dtype))
    return pos.shape[1]


def _check_vec(t: torch.Tensor, n: int, dtype, name: str):
    if not t.is_cuda or t.dtype != dtype or t.shape != (n,) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor of shape [%d]" % (name, dtype, n))


def force(pos: torch.Tensor, mass: torch.Tensor, eps: float, precision: str = "comp",
          with_pot: bool = True, out=None, **kw):
    """Accelerations ``[3, n]`` (float64) and potentials ``[n]`` (float64, or None)."""
    n = _check_pos(pos, torch.float32)
    _check_vec(mass, n, torch.float32, "mass")
    acc, pot = out if out is not None else (
        torch.empty((3, n), dtype=torch.float64, device=pos.device),
        torch.empty(n, dtype=torch.float64, device=pos.device) if with_pot else None)
    opts = make_opts(precision=precision, **kw)
    _lib.nbody_force_ex(n, pos.data_ptr(), mass.data_ptr(), float(eps), acc.data_ptr(),
                        pot.data_ptr() if pot is not None else None, opts, stream_ptr())
    return acc, pot


def force_f64(pos64: torch.Tensor, mass: torch.Tensor, eps: float, precision: str = "comp",
              centre: str = "system", with_pot: bool = True, out=None, **kw):
    """As ``force`` for float64 positions taken relative to a reference centre."""
    n = _check_pos(pos64, torch.float64, "pos64")
    _check_vec(mass, n, torch.float32, "mass")
    acc, pot = out if out is not None else (
        torch.empty((3, n), dtype=torch.float64, device=pos64.device),
        torch.empty(n, dtype=torch.float64, device=pos64.device) if with_pot else None)
    opts = make_opts(precision=precision, centre=centre, **kw)
    _lib.nbody_force_f64(n, pos64.data_ptr(), mass.data_ptr(), float(eps), acc.data_ptr(),
                         pot.data_ptr() if pot is not None else None, opts, stream_ptr())
    return acc, pot


def force_ij(pos_i: torch.Tensor, pos_j: torch.Tensor, mass_j: torch.Tensor, eps: float = 0.0,
             eps_i: torch.Tensor | None = None, precision: str = "comp", with_pot: bool = True,
             out=None, **kw):
    """Accelerations ``[3, ni]`` and potentials ``[ni]`` (float64) on the i-set from the
    j-set; every pair counts (no self pair).  ``eps_i`` (float32 ``[ni]``) gives a
    softening per i-particle instead of the uniform ``eps``."""
    ni = _check_pos(pos_i, torch.float32, "pos_i")
    nj = _check_pos(pos_j, torch.float32, "pos_j")
    _check_vec(mass_j, nj, torch.float32, "mass_j")
    if eps_i is not None:
        _check_vec(eps_i, ni, torch.float32, "eps_i")
    acc, pot = out if out is not None else (
        torch.empty((3, ni), dtype=torch.float64, device=pos_i.device),
        torch.empty(ni, dtype=torch.float64, device=pos_i.device) if with_pot else None)
    opts = make_opts(precision=precision, **kw)
    _lib.nbody_force_ij(ni, pos_i.data_ptr(), eps_i.data_ptr() if eps_i is not None else None,
                        nj, pos_j.data_ptr(), mass_j.data_ptr(), float(eps), acc.data_ptr(),
                        pot.data_ptr() if pot is not None else None, opts, stream_ptr())
    return acc, pot


def force_jerk(pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, eps: float,
               precision: str = "comp", with_pot: bool = True, out=None, **kw):
    """``(acc, jerk, pot)``: accelerations and jerks ``[3, n]`` and potentials ``[n]``
    (float64) from float32 (``[3, n]``) or float64 state; float64 state is taken relative
    to its mean position and velocity (``centre="system"``) or just rounded
    (``centre="none"``)."""
    f64 = pos.dtype == torch.float64
    n = _check_pos(pos, torch.float64 if f64 else torch.float32)
    if _check_pos(vel, pos.dtype, "vel") != n:
        raise ValueError("vel must have the shape of pos")
    _check_vec(mass, n, torch.float32, "mass")
    dev = pos.device
    acc, jerk, pot = out if out is not None else (
        torch.empty((3, n), dtype=torch.float64, device=dev),
        torch.empty((3, n), dtype=torch.float64, device=dev),
        torch.empty(n, dtype=torch.float64, device=dev) if with_pot else None)
    opts = make_opts(precision=precision, **kw)
    fn = _lib.nbody_force_jerk_f64 if f64 else _lib.nbody_force_jerk
    fn(n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), float(eps), acc.data_ptr(),
       jerk.data_ptr(), pot.data_ptr() if pot is not None else None, opts, stream_ptr())
    return acc, jerk, pot


def force_jerk_ij(pos_i: torch.Tensor, vel_i: torch.Tensor, pos_j: torch.Tensor,
                  vel_j: torch.Tensor, mass_j: torch.Tensor, eps: float = 0.0,
                  precision: str = "comp", with_pot: bool = True, out=None, **kw):
    """``(acc, jerk, pot)`` (float64, ``[3, ni]``, ``[3, ni]``, ``[ni]``) on the i-set from
    the j-set, float32 ``[3, n]`` inputs; every pair counts (no self pair)."""
    ni = _check_pos(pos_i, torch.float32, "pos_i")
    if _check_pos(vel_i, torch.float32, "vel_i") != ni:
        raise ValueError("vel_i must have the shape of pos_i")
    nj = _check_pos(pos_j, torch.float32, "pos_j")
    if _check_pos(vel_j, torch.float32, "vel_j") != nj:
        raise ValueError("vel_j must have the shape of pos_j")
    _check_vec(mass_j, nj, torch.float32, "mass_j")
    dev = pos_i.device
    acc, jerk, pot = out if out is not None else (
        torch.empty((3, ni), dtype=torch.float64, device=dev),
        torch.empty((3, ni), dtype=torch.float64, device=dev),
        torch.empty(ni, dtype=torch.float64, device=dev) if with_pot else None)
    opts = make_opts(precision=precision, **kw)
    _lib.nbody_force_jerk_ij(ni, pos_i.data_ptr(), vel_i.data_ptr(), nj, pos_j.data_ptr(),
                             vel_j.data_ptr(), mass_j.data_ptr(), float(eps), acc.data_ptr(),
                             jerk.data_ptr(), pot.data_ptr() if pot is not None else None, opts,
                             stream_ptr())
    return acc, jerk, pot


def morton_order(pos64: torch.Tensor) -> torch.Tensor:
    """int32 permutation ``[n]`` ordering the particles along the Z-curve."""
    n = _check_pos(pos64, torch.float64, "pos64")
    perm = torch.empty(n, dtype=torch.int32, device=pos64.device)
    _lib.nbody_morton_order(n, pos64.data_ptr(), perm.data_ptr(), stream_ptr())
    return perm


def leapfrog(pos64: torch.Tensor, vel64: torch.Tensor, mass: torch.Tensor, eps: float, dt: float,
             nsteps: int, acc: torch.Tensor | None = None, init: bool = True,
             with_pot: bool = False, keep_trajectory: bool = False, precision: str = "comp",
             centre: str = "system", **kw):
    """``nsteps`` KDK steps on ``pos64``/``vel64`` in place.

    Returns ``(acc, pot, traj)``: a(x) at the final positions ``[3, n]``, the final
    potentials (or None) and the position checkpoints ``[nsteps + 1, 3, n]`` (or None).
    With ``init=False`` ``acc`` must already hold a(pos64).
    """
    n = _check_pos(pos64, torch.float64, "pos64")
    _check_pos(vel64, torch.float64, "vel64")
    _check_vec(mass, n, torch.float32, "mass")
    dev = pos64.device
    if acc is None:
        if not init:
            raise ValueError("acc is required when init=False")
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev) if with_pot else None
    traj = (torch.empty((nsteps + 1, 3, n), dtype=torch.float64, device=dev)
            if keep_trajectory else None)
    opts = make_opts(precision=precision, centre=centre, **kw)
    _lib.nbody_leapfrog(n, pos64.data_ptr(), vel64.data_ptr(), mass.data_ptr(), float(eps),
                        float(dt), int(nsteps), acc.data_ptr(),
                        pot.data_ptr() if pot is not None else None,
                        traj.data_ptr() if traj is not None else None,
                        _lib.NBODY_LF_INIT_ACC if init else 0, opts, stream_ptr())
    return acc, pot, traj


class LeapfrogGraph:
    """A HIP graph of ``nsteps`` KDK steps on fixed tensors (replayed by ``launch``).

    The tensors are referenced, not copied: keep them alive and update them in place.
    ``acc`` must hold a(pos64) before the first launch.
    """

    def __init__(self, pos64, vel64, mass, eps, dt, nsteps, acc, pot=None, precision="comp",
                 centre="system", **kw):
        n = _check_pos(pos64, torch.float64, "pos64")
        _check_pos(vel64, torch.float64, "vel64")
        _check_pos(acc, torch.float64, "acc")
        _check_vec(mass, n, torch.float32, "mass")
        self._keep = (pos64, vel64, mass, acc, pot)
        opts = make_opts(precision=precision, centre=centre, **kw)
        self.handle = _lib.nbody_graph_create_leapfrog(
            n, pos64.data_ptr(), vel64.data_ptr(), mass.data_ptr(), float(eps), float(dt),
            int(nsteps), acc.data_ptr(), pot.data_ptr() if pot is not None else None, opts,
            stream_ptr())

    def launch(self, stream: torch.cuda.Stream | None = None):
        _lib.nbody_graph_launch(self.handle, stream_ptr(stream))

    def close(self):
        if self.handle:
            _lib.nbody_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hermite(pos64: torch.Tensor, vel64: torch.Tensor, mass: torch.Tensor, eps: float, dt: float,
            nsteps: int, acc: torch.Tensor | None = None, jerk: torch.Tensor | None = None,
            init: bool = True, precision: str = "comp", centre: str = "system", **kw):
    """``nsteps`` fourth-order Hermite steps on ``pos64``/``vel64`` in place.

    Returns ``(acc, jerk)`` of the last evaluation ``[3, n]``; with ``init=False`` they
    must hold a and j at the entry state (as returned by a previous call).
    """
    n = _check_pos(pos64, torch.float64, "pos64")
    _check_pos(vel64, torch.float64, "vel64")
    _check_vec(mass, n, torch.float32, "mass")
    dev = pos64.device
    if acc is None:
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    if jerk is None:
        jerk = torch.empty((3, n), dtype=torch.float64, device=dev)
    opts = make_opts(precision=precision, centre=centre, **kw)
    _lib.nbody_hermite(n, pos64.data_ptr(), vel64.data_ptr(), mass.data_ptr(), float(eps),
                       float(dt), int(nsteps), acc.data_ptr(), jerk.data_ptr(),
                       _lib.NBODY_LF_INIT_ACC if init else 0, opts, stream_ptr())
    return acc, jerk


class HermiteGraph(LeapfrogGraph):
    """A HIP graph of ``nsteps`` Hermite steps on fixed tensors (replayed by ``launch``);
    ``acc`` and ``jerk`` must hold a and j at the state before the first launch."""

    def __init__(self, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, precision="comp",
                 centre="system", **kw):
        n = _check_pos(pos64, torch.float64, "pos64")
        _check_pos(vel64, torch.float64, "vel64")
        _check_pos(acc, torch.float64, "acc")
        _check_pos(jerk, torch.float64, "jerk")
        _check_vec(mass, n, torch.float32, "mass")
        self._keep = (pos64, vel64, mass, acc, jerk)
        opts = make_opts(precision=precision, centre=centre, **kw)
        self.handle = _lib.nbody_graph_create_hermite(
            n, pos64.data_ptr(), vel64.data_ptr(), mass.data_ptr(), float(eps), float(dt),
            int(nsteps), acc.data_ptr(), jerk.data_ptr(), opts, stream_ptr())


class BatchPlan:
    """Plan for a ragged batch of independent systems (see ``nbody_plan_create_batched``).

    ``offsets``: host sequence of ``nsys + 1`` integers; system k owns the particles
    ``offsets[k]:offsets[k+1]`` of every ``[3, total]`` / ``[total]`` tensor.
    """

    def __init__(self, offsets, precision="comp", centre="system", ipl=0, jtile=0):
        offsets = [int(v) for v in offsets]
        self.nsys = len(offsets) - 1
        self.total = offsets[-1] if offsets else 0
        opts = make_opts(precision=precision, centre=centre, ipl=ipl, jtile=jtile)
        self.handle = _lib.nbody_plan_create_batched(self.nsys, offsets, opts)

    def info(self) -> dict:
        return _lib.nbody_plan_info(self.handle)

    def _out(self, dev, with_pot):
        return (torch.empty((3, self.total), dtype=torch.float64, device=dev),
                torch.empty(self.total, dtype=torch.float64, device=dev) if with_pot else None)

    def force(self, pos, mass, eps, with_pot=True):
        """FP32 positions ``[3, total]``, masses ``[total]``, per-system eps ``[nsys]``."""
        acc, pot = self._out(pos.device, with_pot)
        _lib.nbody_force_batched(self.handle, pos.data_ptr(), mass.data_ptr(), eps.data_ptr(),
                                 acc.data_ptr(), pot.data_ptr() if pot is not None else None,
                                 stream_ptr())
        return acc, pot

    def force_f64(self, pos64, mass, eps, with_pot=True):
        acc, pot = self._out(pos64.device, with_pot)
        _lib.nbody_force_batched_f64(self.handle, pos64.data_ptr(), mass.data_ptr(),
                                     eps.data_ptr(), acc.data_ptr(),
                                     pot.data_ptr() if pot is not None else None, stream_ptr())
        return acc, pot

    def leapfrog(self, pos64, vel64, mass, eps, dt, nsteps, acc=None, init=True, with_pot=False):
        if acc is None:
            acc = torch.empty((3, self.total), dtype=torch.float64, device=pos64.device)
        pot = (torch.empty(self.total, dtype=torch.float64, device=pos64.device)
               if with_pot else None)
        _lib.nbody_leapfrog_batched(self.handle, pos64.data_ptr(), vel64.data_ptr(),
                                    mass.data_ptr(), eps.data_ptr(), float(dt), int(nsteps),
                                    acc.data_ptr(), pot.data_ptr() if pot is not None else None,
                                    _lib.NBODY_LF_INIT_ACC if init else 0, stream_ptr())
        return acc, pot

    def graph(self, pos64, vel64, mass, eps, dt, nsteps, acc, pot=None):
        """A replayable graph of ``nsteps`` batched KDK steps on these tensors."""
        return _BatchGraph(self, pos64, vel64, mass, eps, dt, nsteps, acc, pot)

    def close(self):
        if self.handle:
            _lib.nbody_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _BatchGraph(LeapfrogGraph):
    def __init__(self, plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot):  # noqa: D401
        self._keep = (plan, pos64, vel64, mass, eps, acc, pot)
        self.handle = _lib.nbody_graph_create_leapfrog_batched(
            plan.handle, pos64.data_ptr(), vel64.data_ptr(), mass.data_ptr(), eps.data_ptr(),
            float(dt), int(nsteps), acc.data_ptr(), pot.data_ptr() if pot is not None else None,
            stream_ptr())
