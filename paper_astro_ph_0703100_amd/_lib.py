"""ctypes binding of ``libnbody.so`` with the C function names of ``include/nbody.h``.

Argument marshalling only: every function here forwards plain integers, floats
and device addresses to the C ABI and returns its status.  The library is loaded
on first use; if it has not been built this raises (there is no fallback).

The calls are asynchronous on the given stream and read and write the arrays
behind the addresses later.  A caller passing ``tensor.data_ptr()`` must hold a
reference to every such tensor until the call has returned: a temporary
(``t.float().data_ptr()`` inside the argument list) can be freed, and its memory
handed to the next allocation, before the library has even enqueued its kernels.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnbody.so")

NBODY_OK = 0
NBODY_EINVAL = -1
NBODY_ENOMEM = -2
NBODY_EHIP = -3
NBODY_ECAPTURE = -4
NBODY_EUNSUPPORTED = -5

NBODY_PLAIN = 0
NBODY_FP64RED = 1
NBODY_COMP = 2

NBODY_CENTRE_NONE = 0
NBODY_CENTRE_SYSTEM = 1
NBODY_CENTRE_TILE = 2

PRECISIONS = {"plain": NBODY_PLAIN, "fp64red": NBODY_FP64RED, "comp": NBODY_COMP}
CENTRES = {"none": NBODY_CENTRE_NONE, "system": NBODY_CENTRE_SYSTEM, "tile": NBODY_CENTRE_TILE}


class nbody_opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("centre", ctypes.c_int32),
        ("self_pot", ctypes.c_int32),
        ("ipl", ctypes.c_int32),
        ("jtile", ctypes.c_int32),
        ("nseg", ctypes.c_int32),
        ("jlanes", ctypes.c_int32),
        ("symmetric", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class NBodyError(RuntimeError):
    """A negative status from the library, with its message."""

    def __init__(self, status: int, func: str, msg: str):
        super().__init__("%s failed (status %d): %s" % (func, status, msg))
        self.status = status


_lock = threading.RLock()
_lib = None

_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_P = ctypes.c_void_p
_F = ctypes.c_float
_D = ctypes.c_double
_OPTS = ctypes.POINTER(nbody_opts)

# name -> (restype, argtypes); every symbol include/nbody.h declares.
SIGNATURES = {
    "nbody_opts_default": (None, [_OPTS]),
    "nbody_last_error": (ctypes.c_char_p, []),
    "nbody_version": (ctypes.c_char_p, []),
    "nbody_workspace_size": (ctypes.c_size_t, [_I64, _OPTS]),
    "nbody_force": (_I32, [_I64, _P, _P, _F, _P, _P, _P]),
    "nbody_force_ex": (_I32, [_I64, _P, _P, _F, _P, _P, _OPTS, _P]),
    "nbody_force_f64": (_I32, [_I64, _P, _P, _F, _P, _P, _OPTS, _P]),
    "nbody_force_noalloc": (_I32, [_I64, _P, _P, _F, _P, _P, _OPTS, _P]),
    "nbody_force_ij": (_I32, [_I64, _P, _P, _I64, _P, _P, _F, _P, _P, _OPTS, _P]),
    "nbody_workspace_size_ij": (ctypes.c_size_t, [_I64, _I64, _OPTS]),
    "nbody_force_jerk": (_I32, [_I64, _P, _P, _P, _F, _P, _P, _P, _OPTS, _P]),
    "nbody_force_jerk_ij": (_I32, [_I64, _P, _P, _I64, _P, _P, _P, _F, _P, _P, _P, _OPTS, _P]),
    "nbody_workspace_size_jerk_ij": (ctypes.c_size_t, [_I64, _I64, _OPTS]),
    "nbody_force_jerk_f64": (_I32, [_I64, _P, _P, _P, _F, _P, _P, _P, _OPTS, _P]),
    "nbody_workspace_size_jerk": (ctypes.c_size_t, [_I64, _OPTS]),
    "nbody_hermite": (_I32, [_I64, _P, _P, _P, _F, _D, _I32, _P, _P, _I32, _OPTS, _P]),
    "nbody_graph_create_hermite": (_I32, [_I64, _P, _P, _P, _F, _D, _I32, _P, _P, _OPTS, _P,
                                          ctypes.POINTER(_P)]),
    "nbody_workspace_size_hermite": (ctypes.c_size_t, [_I64, _OPTS]),
    "nbody_leapfrog": (_I32, [_I64, _P, _P, _P, _F, _D, _I32, _P, _P, _P, _I32, _OPTS, _P]),
    "nbody_graph_create_leapfrog": (_I32, [_I64, _P, _P, _P, _F, _D, _I32, _P, _P, _OPTS, _P,
                                           ctypes.POINTER(_P)]),
    "nbody_graph_launch": (_I32, [_P, _P]),
    "nbody_graph_destroy": (None, [_P]),
    "nbody_force_vjp": (_I32, [_I64, _P, _P, _F, _P, _P, _P, _P, _OPTS, _P]),
    "nbody_force_vjp_f64": (_I32, [_I64, _P, _P, _F, _P, _P, _P, _P, _OPTS, _P]),
    "nbody_leapfrog_adjoint": (_I32, [_I64, _P, _P, _F, _D, _I32, _P, _P, _P, _OPTS, _P]),
    "nbody_workspace_size_vjp": (ctypes.c_size_t, [_I64, _OPTS]),
    "nbody_workspace_size_adjoint": (ctypes.c_size_t, [_I64, _OPTS]),
    "nbody_plan_create_batched": (_I32, [_I32, ctypes.POINTER(_I64), _OPTS, ctypes.POINTER(_P)]),
    "nbody_plan_destroy": (None, [_P]),
    "nbody_plan_info": (_I32, [_P, ctypes.POINTER(_I64)]),
    "nbody_force_batched": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "nbody_force_batched_f64": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "nbody_leapfrog_batched": (_I32, [_P, _P, _P, _P, _P, _D, _I32, _P, _P, _I32, _P]),
    "nbody_graph_create_leapfrog_batched": (_I32, [_P, _P, _P, _P, _P, _D, _I32, _P, _P, _P,
                                                   ctypes.POINTER(_P)]),
    "nbody_morton_order": (_I32, [_I64, _P, _P, _P]),
    "nbody_tune_set": (_I32, [_I32, _I32, _I64, _I32, _I32, _I32, _I32, _I32]),
    "nbody_tune_get": (_I32, [_I32, _I32, _I64, ctypes.POINTER(_I32)]),
    "nbody_tune_load": (_I32, [ctypes.c_char_p]),
    "nbody_tune_save": (_I32, [ctypes.c_char_p]),
    "nbody_tune_reset": (None, []),
}

NBODY_KERNEL_FORCE = 0
NBODY_KERNEL_VJP = 1
NBODY_KERNEL_BATCHED = 2
NBODY_KERNEL_JERK = 3
KERNELS = {"force": NBODY_KERNEL_FORCE, "vjp": NBODY_KERNEL_VJP, "batched": NBODY_KERNEL_BATCHED,
           "jerk": NBODY_KERNEL_JERK}
# Tuning table shipped with the package (measured on MI355X by tune.py); loaded with
# the library when present.
TUNING_PATH = os.path.join(_PKG, "tuning_gfx950.json")

NBODY_LF_INIT_ACC = 1


def load():
    """Load ``libnbody.so`` (built in-tree) and declare its functions."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libnbody.so is not built (%s); run python -m paper_astro_ph_0703100_amd.build"
                    % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
            path = os.environ.get("NBODY_TUNING_FILE", TUNING_PATH)
            if path and os.path.exists(path):
                _check(lib.nbody_tune_load(path.encode()), "nbody_tune_load")
    return _lib


def _check(status: int, func: str) -> int:
    if status != NBODY_OK:
        raise NBodyError(status, func, nbody_last_error())
    return status


def nbody_last_error() -> str:
    return load().nbody_last_error().decode()


def nbody_version() -> str:
    return load().nbody_version().decode()


def nbody_opts_default() -> nbody_opts:
    o = nbody_opts()
    load().nbody_opts_default(ctypes.byref(o))
    return o


def nbody_workspace_size(n: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size(n, ctypes.byref(opts) if opts is not None else None))


def nbody_force(n, pos, mass, eps, acc, pot, stream, check=True):
    st = load().nbody_force(n, pos, mass, eps, acc, pot, stream)
    return _check(st, "nbody_force") if check else st


def nbody_force_ex(n, pos, mass, eps, acc, pot, opts, stream, check=True):
    st = load().nbody_force_ex(n, pos, mass, eps, acc, pot,
                               ctypes.byref(opts) if opts is not None else None, stream)
    return _check(st, "nbody_force_ex") if check else st


def nbody_force_f64(n, pos64, mass, eps, acc, pot, opts, stream, check=True):
    st = load().nbody_force_f64(n, pos64, mass, eps, acc, pot,
                                ctypes.byref(opts) if opts is not None else None, stream)
    return _check(st, "nbody_force_f64") if check else st


NBODY_NOALLOC_SCRATCH_BYTES = 64 << 20


def nbody_force_noalloc(n, pos, mass, eps, acc, pot, opts, stream, check=True):
    st = load().nbody_force_noalloc(n, pos, mass, eps, acc, pot,
                                    ctypes.byref(opts) if opts is not None else None, stream)
    return _check(st, "nbody_force_noalloc") if check else st


def nbody_force_ij(ni, pos_i, eps_i, nj, pos_j, mass_j, eps, acc, pot, opts, stream, check=True):
    st = load().nbody_force_ij(ni, pos_i, eps_i, nj, pos_j, mass_j, eps, acc, pot,
                               ctypes.byref(opts) if opts is not None else None, stream)
    return _check(st, "nbody_force_ij") if check else st


def nbody_workspace_size_ij(ni: int, nj: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_ij(ni, nj, ctypes.byref(opts) if opts is not None
                                              else None))


def nbody_force_jerk(n, pos, vel, mass, eps, acc, jerk, pot, opts, stream, check=True):
    st = load().nbody_force_jerk(n, pos, vel, mass, eps, acc, jerk, pot, _opt_ref(opts), stream)
    return _check(st, "nbody_force_jerk") if check else st


def nbody_force_jerk_f64(n, pos64, vel64, mass, eps, acc, jerk, pot, opts, stream, check=True):
    st = load().nbody_force_jerk_f64(n, pos64, vel64, mass, eps, acc, jerk, pot, _opt_ref(opts),
                                     stream)
    return _check(st, "nbody_force_jerk_f64") if check else st


def nbody_force_jerk_ij(ni, pos_i, vel_i, nj, pos_j, vel_j, mass_j, eps, acc, jerk, pot, opts,
                        stream, check=True):
    st = load().nbody_force_jerk_ij(ni, pos_i, vel_i, nj, pos_j, vel_j, mass_j, eps, acc, jerk,
                                    pot, _opt_ref(opts), stream)
    return _check(st, "nbody_force_jerk_ij") if check else st


def nbody_workspace_size_jerk_ij(ni: int, nj: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_jerk_ij(ni, nj, _opt_ref(opts)))


def nbody_workspace_size_jerk(n: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_jerk(n, _opt_ref(opts)))


def nbody_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, flags, opts, stream,
                  check=True):
    st = load().nbody_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, flags,
                              _opt_ref(opts), stream)
    return _check(st, "nbody_hermite") if check else st


def nbody_graph_create_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, opts, stream):
    """Returns the graph handle (an integer address)."""
    h = ctypes.c_void_p()
    st = load().nbody_graph_create_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk,
                                           _opt_ref(opts), stream, ctypes.byref(h))
    _check(st, "nbody_graph_create_hermite")
    return h.value


def nbody_workspace_size_hermite(n: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_hermite(n, _opt_ref(opts)))


def nbody_workspace_size_vjp(n: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_vjp(n, _opt_ref(opts)))


def nbody_workspace_size_adjoint(n: int, opts: nbody_opts | None) -> int:
    return int(load().nbody_workspace_size_adjoint(n, _opt_ref(opts)))


def _opt_ref(opts):
    return ctypes.byref(opts) if opts is not None else None


def nbody_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot, traj, flags, opts, stream,
                   check=True):
    st = load().nbody_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot, traj, flags,
                               _opt_ref(opts), stream)
    return _check(st, "nbody_leapfrog") if check else st


def nbody_graph_create_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot, opts, stream):
    """Returns the graph handle (an integer address)."""
    h = ctypes.c_void_p()
    st = load().nbody_graph_create_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot,
                                            _opt_ref(opts), stream, ctypes.byref(h))
    _check(st, "nbody_graph_create_leapfrog")
    return h.value


def nbody_graph_launch(graph, stream, check=True):
    st = load().nbody_graph_launch(graph, stream)
    return _check(st, "nbody_graph_launch") if check else st


def nbody_graph_destroy(graph):
    load().nbody_graph_destroy(graph)


def nbody_force_vjp(n, pos, mass, eps, g_acc, g_pot, grad_pos, grad_mass, opts, stream,
                    check=True):
    st = load().nbody_force_vjp(n, pos, mass, eps, g_acc, g_pot, grad_pos, grad_mass,
                                _opt_ref(opts), stream)
    return _check(st, "nbody_force_vjp") if check else st


def nbody_force_vjp_f64(n, pos64, mass, eps, g_acc, g_pot, grad_pos, grad_mass, opts, stream,
                        check=True):
    st = load().nbody_force_vjp_f64(n, pos64, mass, eps, g_acc, g_pot, grad_pos, grad_mass,
                                    _opt_ref(opts), stream)
    return _check(st, "nbody_force_vjp_f64") if check else st


def nbody_leapfrog_adjoint(n, traj, mass, eps, dt, nsteps, xbar, vbar, mbar, opts, stream,
                           check=True):
    st = load().nbody_leapfrog_adjoint(n, traj, mass, eps, dt, nsteps, xbar, vbar, mbar,
                                       _opt_ref(opts), stream)
    return _check(st, "nbody_leapfrog_adjoint") if check else st


def nbody_plan_create_batched(nsys, offsets, opts):
    """``offsets``: sequence of nsys + 1 host integers.  Returns the plan handle."""
    arr = (_I64 * (nsys + 1))(*[int(v) for v in offsets])
    h = ctypes.c_void_p()
    st = load().nbody_plan_create_batched(nsys, arr, _opt_ref(opts), ctypes.byref(h))
    _check(st, "nbody_plan_create_batched")
    return h.value


def nbody_plan_destroy(plan):
    load().nbody_plan_destroy(plan)


def nbody_plan_info(plan):
    info = (_I64 * 8)()
    _check(load().nbody_plan_info(plan, info), "nbody_plan_info")
    keys = ("nsys", "total", "items", "blocks", "pairs", "padded_pairs", "ipl", "jtile")
    return dict(zip(keys, [int(v) for v in info]))


def nbody_force_batched(plan, pos, mass, eps, acc, pot, stream, check=True):
    st = load().nbody_force_batched(plan, pos, mass, eps, acc, pot, stream)
    return _check(st, "nbody_force_batched") if check else st


def nbody_force_batched_f64(plan, pos64, mass, eps, acc, pot, stream, check=True):
    st = load().nbody_force_batched_f64(plan, pos64, mass, eps, acc, pot, stream)
    return _check(st, "nbody_force_batched_f64") if check else st


def nbody_leapfrog_batched(plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot, flags, stream,
                           check=True):
    st = load().nbody_leapfrog_batched(plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot, flags,
                                       stream)
    return _check(st, "nbody_leapfrog_batched") if check else st


def nbody_graph_create_leapfrog_batched(plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot,
                                        stream):
    h = ctypes.c_void_p()
    st = load().nbody_graph_create_leapfrog_batched(plan, pos64, vel64, mass, eps, dt, nsteps,
                                                    acc, pot, stream, ctypes.byref(h))
    _check(st, "nbody_graph_create_leapfrog_batched")
    return h.value


def nbody_tune_set(kernel, precision, n, ipl, jtile, nseg, jlanes=1, symmetric=0):
    return _check(load().nbody_tune_set(kernel, precision, n, ipl, jtile, nseg, jlanes, symmetric),
                  "nbody_tune_set")


def nbody_tune_get(kernel, precision, n):
    """(ipl, jtile, nseg, jlanes, symmetric) in effect for (kernel, precision, n)."""
    shape = (_I32 * 5)()
    _check(load().nbody_tune_get(kernel, precision, n, shape), "nbody_tune_get")
    return tuple(int(v) for v in shape)


def nbody_tune_load(path):
    return _check(load().nbody_tune_load(str(path).encode()), "nbody_tune_load")


def nbody_tune_save(path):
    return _check(load().nbody_tune_save(str(path).encode()), "nbody_tune_save")


def nbody_tune_reset():
    load().nbody_tune_reset()


def nbody_morton_order(n, pos64, perm, stream, check=True):
    st = load().nbody_morton_order(n, pos64, perm, stream)
    return _check(st, "nbody_morton_order") if check else st
