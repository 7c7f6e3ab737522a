"""Torch-tensor front end of the C ABI (argument marshalling only).

Tensors are device tensors in the library's layout: positions ``[3, n]``
(structure of arrays), masses ``[n]``.  Outputs are allocated here with
``torch.empty`` and filled by the library on the current HIP stream; nothing is
computed in torch.
"""
from __future__ import annotations

import torch

from . import _lib

__all__ = ["make_opts", "force", "force_f64", "soa", "aos", "stream_ptr"]


def make_opts(precision: str = "comp", centre: str = "system", self_pot: bool = False,
              ipl: int = 0, jtile: int = 0, nseg: int = 0, workspace: torch.Tensor | None = None):
    o = _lib.nbody_opts_default()
    o.precision = _lib.PRECISIONS[precision]
    o.centre = _lib.CENTRES[centre]
    o.self_pot = int(bool(self_pot))
    o.ipl, o.jtile, o.nseg = int(ipl), int(jtile), int(nseg)
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
