"""Plain FP64 CPU oracle for softened direct-sum gravity (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library and imports nothing from it.
The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64, IEEE sqrt and
division); this module builds it with gcc and wraps it with ctypes over numpy
arrays.  Positions are ``(n, 3)`` float64 arrays, masses ``(n,)`` float64.

Parity status of each function (what pins it; the pins are in tests/test_oracle.py):
  force_all / force_sampled / force_ij : two-body closed form, 50-digit brute
      force, momentum conservation, Plummer mean field, exact power-of-two
      scaling, coincident pair, n = 1, permutation, Table 2 error magnitudes.
  force_ij with eps_i : two-body closed forms with a different softening per
      i-particle (including eps = 0), 50-digit brute force on separate i- and
      j-sets with per-i softening.
  force_abs           : equals |a_c| and |phi| (from the pinned force functions) for
      positive masses lying on one side of every i along each axis; otherwise it
      bounds them; it is the same pair set as force_ij / force_sampled.
  force_jerk          : two-body closed form, central time differences of
      force_all along x + v t, 50-digit brute force, sum_i m_i jerk_i = 0,
      exact power-of-two scaling of v, Galilean invariance.
  force_jerk_ij       : central time differences of the (pinned) force_ij along
      straight-line motion of both sets; on i-set = j-set it equals force_jerk
      exactly in a and the jerk, and in phi up to the self term -m_i/eps.
  vjp                 : central finite differences of force_all, translation
      invariance, degree-1 homogeneity in the masses.
  rollout             : time reversibility, second-order energy error, two-body
      circular orbit.
  rollout_loss_grad   : central finite differences of the rollout loss (n = 12, and
      at the full N = 16384, 32-step differentiation workload in a slow test).
  rollout_vjp         : central finite differences of a loss on both final positions
      and final velocities, zero steps (identity) and one step included.
  hermite             : two-body circular orbit with fourth-order phase error,
      fourth-order energy error, agreement with the (pinned) leapfrog at a much
      smaller step, exact free motion.
  fp32_replay         : the paper's Table 2 magnitudes (order of magnitude only).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_L = ctypes.POINTER(ctypes.c_int64)
_I64 = ctypes.c_int64


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_force.argtypes = [_I64, _D, _D, _I64, _D, _L, ctypes.c_double, _D, _D]
            lib.oracle_hermite.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                           _I64, _D, _D]
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_force_epsi.argtypes = [_I64, _D, _D, _I64, _D, _D, _D, _D]
            lib.oracle_force_abs.argtypes = [_I64, _D, _D, _I64, _D, _L, ctypes.c_double, _D, _D]
            lib.oracle_force_abs.restype = None
            lib.oracle_force_jerk.argtypes = [_I64, _D, _D, _D, _I64, _D, _D, _L, ctypes.c_double,
                                              _D, _D, _D]
            lib.oracle_force_all.argtypes = [_I64, _D, _D, ctypes.c_double, _D, _D]
            lib.oracle_force_sampled.argtypes = [_I64, _D, _D, ctypes.c_double, _I64, _L, _D, _D]
            lib.oracle_vjp.argtypes = [_I64, _D, _D, ctypes.c_double, _D, _D, _D, _D]
            lib.oracle_rollout.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                           _I64, _D, _D]
            lib.oracle_rollout_loss_grad.argtypes = [_I64, _D, _D, _D, ctypes.c_double,
                                                     ctypes.c_double, _I64, _D, _D, _D, _D]
            lib.oracle_rollout_loss_grad.restype = ctypes.c_double
            lib.oracle_rollout_vjp.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                               _I64, _D, _D, _D, _D, _D]
            lib.oracle_rollout_vjp.restype = None
            lib.oracle_fp32_replay.argtypes = [_I64, _F, _F, ctypes.c_float, _I64, _I64, _L, _D]
            lib.oracle_threads.restype = ctypes.c_int
            for f in (lib.oracle_force, lib.oracle_force_all, lib.oracle_force_sampled,
                      lib.oracle_vjp, lib.oracle_rollout, lib.oracle_fp32_replay):
                f.restype = None
            _lib = lib
    return _lib


def _p(a, ptype=_D):
    return None if a is None else a.ctypes.data_as(ptype)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def threads() -> int:
    """OpenMP threads the oracle runs with (``OMP_NUM_THREADS`` or all host threads)."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> int:
    """Run the oracle on ``n`` OpenMP threads from now on; returns the previous count."""
    lib = _load()
    old = int(lib.oracle_threads())
    lib.oracle_set_threads(int(n))
    return old


def force_all(x, m, eps):
    """(acc (n,3), pot (n,)) of every particle from all others, self pair excluded."""
    x = _f64(x)
    n = x.shape[0]
    m = _f64(m, (n,))
    acc = np.empty((n, 3))
    pot = np.empty(n)
    _load().oracle_force_all(n, _p(x), _p(m), float(eps), _p(acc), _p(pot))
    return acc, pot


def force_sampled(x, m, eps, idx):
    """(acc (k,3), pot (k,)) of the particles ``idx`` from all n particles, self excluded."""
    x = _f64(x)
    n = x.shape[0]
    m = _f64(m, (n,))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("sample index out of range")
    k = idx.size
    acc = np.empty((k, 3))
    pot = np.empty(k)
    _load().oracle_force_sampled(n, _p(x), _p(m), float(eps), k, _p(idx, _L), _p(acc), _p(pot))
    return acc, pot


def force_ij(xj, mj, xi, eps, self_index=None, eps_i=None):
    """Forces on separate i-particles ``xi`` from j-particles (``xj``, ``mj``).

    ``self_index[i]`` names a j to leave out for i (or -1); None leaves none out.
    ``eps_i`` (one softening length per i-particle) replaces ``eps``; it cannot be
    combined with ``self_index``.
    """
    xj = _f64(xj)
    xi = _f64(xi)
    nj, ni = xj.shape[0], xi.shape[0]
    mj = _f64(mj, (nj,))
    if eps_i is not None:
        if self_index is not None:
            raise ValueError("eps_i and self_index cannot be combined")
        ei = _f64(eps_i, (ni,))
        acc = np.empty((ni, 3))
        pot = np.empty(ni)
        _load().oracle_force_epsi(nj, _p(xj), _p(mj), ni, _p(xi), _p(ei), _p(acc), _p(pot))
        return acc, pot
    si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
    acc = np.empty((ni, 3))
    pot = np.empty(ni)
    _load().oracle_force(nj, _p(xj), _p(mj), ni, _p(xi), _p(si, _L), float(eps), _p(acc), _p(pot))
    return acc, pot


def force_abs(xj, mj, xi, eps, self_index=None):
    """Magnitude sums for rounding bounds on the i-particles ``xi`` from the j-set:
    (sum_j |m_j d_c| / s^3 per component (ni, 3), sum_j |m_j| / s (ni,)), skipping
    j = ``self_index[i]`` (None: no pair skipped)."""
    xj = _f64(xj)
    xi = _f64(xi)
    nj, ni = xj.shape[0], xi.shape[0]
    mj = _f64(mj, (nj,))
    si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
    absa, absp = np.empty((ni, 3)), np.empty(ni)
    _load().oracle_force_abs(nj, _p(xj), _p(mj), ni, _p(xi), _p(si, _L), float(eps), _p(absa),
                             _p(absp))
    return absa, absp


def force_abs_sampled(x, m, eps, idx):
    """force_abs of the particles ``idx`` of one set from all of it, self pair skipped."""
    x = _f64(x)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    return force_abs(x, m, x[idx], eps, self_index=idx)


def force_jerk(x, v, m, eps, idx=None):
    """(acc, jerk, pot) of every particle (or of the sampled ``idx``) from all others,
    self pair excluded; ``x``, ``v`` are ``(n, 3)``."""
    x = _f64(x)
    n = x.shape[0]
    v = _f64(v, (n, 3))
    m = _f64(m, (n,))
    if idx is None:
        idx = np.arange(n, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("sample index out of range")
    xi = np.ascontiguousarray(x[idx])
    vi = np.ascontiguousarray(v[idx])
    k = idx.size
    acc, jerk, pot = np.empty((k, 3)), np.empty((k, 3)), np.empty(k)
    _load().oracle_force_jerk(n, _p(x), _p(v), _p(m), k, _p(xi), _p(vi), _p(idx, _L), float(eps),
                              _p(acc), _p(jerk), _p(pot))
    return acc, jerk, pot


def force_jerk_ij(xj, vj, mj, xi, vi, eps):
    """(acc, jerk, pot) on the i-set ``xi``, ``vi`` ``(ni, 3)`` from the j-set; every
    (i, j) pair is summed (no self pair), one softening ``eps`` for all."""
    xj = _f64(xj)
    nj = xj.shape[0]
    vj = _f64(vj, (nj, 3))
    mj = _f64(mj, (nj,))
    xi = _f64(xi)
    ni = xi.shape[0]
    vi = _f64(vi, (ni, 3))
    acc, jerk, pot = np.empty((ni, 3)), np.empty((ni, 3)), np.empty(ni)
    _load().oracle_force_jerk(nj, _p(xj), _p(vj), _p(mj), ni, _p(xi), _p(vi), None, float(eps),
                              _p(acc), _p(jerk), _p(pot))
    return acc, jerk, pot


def vjp(x, m, eps, g_acc, g_pot=None):
    """(grad_x (n,3), grad_m (n,)) of L given dL/da = ``g_acc`` and dL/dphi = ``g_pot``."""
    x = _f64(x)
    n = x.shape[0]
    m = _f64(m, (n,))
    ga = _f64(g_acc, (n, 3))
    gp = None if g_pot is None else _f64(g_pot, (n,))
    gx = np.empty((n, 3))
    gm = np.empty(n)
    _load().oracle_vjp(n, _p(x), _p(m), float(eps), _p(ga), _p(gp), _p(gx), _p(gm))
    return gx, gm


def rollout(x0, v0, m, eps, dt, nsteps, keep_trajectory=False):
    """KDK leapfrog: returns (x_T, v_T, a(x_T), trajectory or None)."""
    x = _f64(x0).copy()
    n = x.shape[0]
    v = _f64(v0, (n, 3)).copy()
    m = _f64(m, (n,))
    traj = np.empty((nsteps + 1, n, 3)) if keep_trajectory else None
    acc = np.empty((n, 3))
    _load().oracle_rollout(n, _p(x), _p(v), _p(m), float(eps), float(dt), int(nsteps),
                           _p(traj), _p(acc))
    return x, v, acc, traj


def hermite(x0, v0, m, eps, dt, nsteps):
    """Fourth-order Hermite (shared step): returns (x_T, v_T, a_T, jerk_T)."""
    x = _f64(x0).copy()
    n = x.shape[0]
    v = _f64(v0, (n, 3)).copy()
    m = _f64(m, (n,))
    acc, jerk = np.empty((n, 3)), np.empty((n, 3))
    _load().oracle_hermite(n, _p(x), _p(v), _p(m), float(eps), float(dt), int(nsteps), _p(acc),
                           _p(jerk))
    return x, v, acc, jerk


def rollout_loss_grad(x0, v0, m, eps, dt, nsteps, target):
    """(L, dL/dx0, dL/dv0, dL/dm) for L = mean_i |x_i(T) - y_i|^2 after ``nsteps`` KDK steps."""
    x0 = _f64(x0)
    n = x0.shape[0]
    v0 = _f64(v0, (n, 3))
    m = _f64(m, (n,))
    y = _f64(target, (n, 3))
    gx = np.empty((n, 3))
    gv = np.empty((n, 3))
    gm = np.empty(n)
    loss = _load().oracle_rollout_loss_grad(n, _p(x0), _p(v0), _p(m), float(eps), float(dt),
                                            int(nsteps), _p(y), _p(gx), _p(gv), _p(gm))
    return float(loss), gx, gv, gm


def rollout_vjp(x0, v0, m, eps, dt, nsteps, xbar_T=None, vbar_T=None):
    """(dL/dx0, dL/dv0, dL/dm) of ``nsteps`` KDK steps for the cotangents ``xbar_T`` =
    dL/dx_T and ``vbar_T`` = dL/dv_T of the final state (``(n, 3)``; None = zero)."""
    x0 = _f64(x0)
    n = x0.shape[0]
    v0 = _f64(v0, (n, 3))
    m = _f64(m, (n,))
    xb = None if xbar_T is None else _f64(xbar_T, (n, 3))
    vb = None if vbar_T is None else _f64(vbar_T, (n, 3))
    gx, gv, gm = np.empty((n, 3)), np.empty((n, 3)), np.empty(n)
    _load().oracle_rollout_vjp(n, _p(x0), _p(v0), _p(m), float(eps), float(dt), int(nsteps),
                               _p(xb), _p(vb), _p(gx), _p(gv), _p(gm))
    return gx, gv, gm


def fp32_replay(x32, m32, eps2_32, nbag, idx):
    """Single-precision replay of the paper's DIRECT (nbag=0) or J-BAG (nbag>0) order."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    n = x32.shape[0]
    m32 = np.ascontiguousarray(m32, dtype=np.float32)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    acc = np.empty((idx.size, 3))
    _load().oracle_fp32_replay(n, _p(x32, _F), _p(m32, _F), float(np.float32(eps2_32)),
                               int(nbag), idx.size, _p(idx, _L), _p(acc))
    return acc


def energy(x, v, m, eps):
    """Total energy sum_i m_i v_i^2 / 2 + sum_i m_i phi_i / 2 (pair potential counted once)."""
    _, pot = force_all(x, m, eps)
    m = _f64(m)
    return float(0.5 * np.sum(m * np.sum(_f64(v) ** 2, axis=1)) + 0.5 * np.sum(m * pot))
