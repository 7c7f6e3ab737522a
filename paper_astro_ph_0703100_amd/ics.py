"""Seeded synthetic initial conditions shared by the tests, the bench and the oracle checks.

This module holds no part of the force computation: it only draws particle sets.
The paper's experiments use an equal-mass Plummer sphere in virial equilibrium
(Sec. 3.3, and the captions of Tables 2 and 3).  The paper built it with an
external toolbox that is not available here, so the sphere is sampled from the
published distribution function of the Plummer model (Aarseth, Henon & Wielen
1974): radius from the inverted cumulative mass profile, isotropic directions,
speed from the distribution function by rejection.  Units are G = M = 1 with
scale radius ``a``.

Every generator takes an explicit integer seed and uses numpy's PCG64
(``numpy.random.default_rng``), so the same seed gives the same particles on
any host.  Positions and velocities come back as float64 arrays of shape
``(n, 3)`` (array of structures), masses as float64 ``(n,)``; callers convert
to the device layout themselves.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "plummer",
    "nemo_plummer",
    "stress_system",
    "cluster_batch",
    "sample_indices",
    "stratified_indices",
    "perturbed_target",
    "plummer_131072_eps",
    "Workload",
    "WORKLOADS",
]


def _plummer_radii(rng: np.random.Generator, n: int, rmax: float) -> np.ndarray:
    """Radii in units of the scale radius, from M(<r) = r^3 / (1 + r^2)^{3/2}.

    Inverting X = M(<r) gives r = (X^{-2/3} - 1)^{-1/2}; draws beyond ``rmax``
    are redrawn, which truncates the sphere at ``rmax`` scale radii.
    """
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.random(todo.size)
        # x == 0 would give r == 0 exactly; that is a valid (if unlikely) draw.
        with np.errstate(divide="ignore"):
            rr = 1.0 / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)
        ok = np.isfinite(rr) & (rr <= rmax)
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    return r


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: cos(theta) uniform in [-1, 1], phi in [0, 2 pi)."""
    ct = 2.0 * rng.random(n) - 1.0
    ph = 2.0 * math.pi * rng.random(n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def _plummer_speed_fraction(rng: np.random.Generator, n: int) -> np.ndarray:
    """q = v / v_esc drawn from g(q) ~ q^2 (1 - q^2)^{7/2} on [0, 1] by rejection.

    The envelope 0.1 bounds g (its maximum is about 0.0922).
    """
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x4 = rng.random(todo.size)
        x5 = rng.random(todo.size)
        ok = 0.1 * x5 < x4 * x4 * np.power(1.0 - x4 * x4, 3.5)
        q[todo[ok]] = x4[ok]
        todo = todo[~ok]
    return q


def plummer(n: int, seed: int, a: float = 1.0, rmax: float = 20.0,
            velocities: bool = True, total_mass: float = 1.0):
    """Equal-mass Plummer sphere of ``n`` particles, total mass ``total_mass``.

    Positions are scaled by ``a``; velocities by sqrt(M / a) (G = 1).  The sphere
    is truncated at ``rmax`` scale radii.  The centre of mass position and velocity
    are removed in float64.  With ``velocities=False`` the velocities are zero.
    Returns ``(pos, vel, mass)``.
    """
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = np.random.default_rng(seed)
    mass = np.full(n, total_mass / n if n else 0.0)
    if n == 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), mass
    r = _plummer_radii(rng, n, rmax)
    pos = r[:, None] * _isotropic(rng, n)
    if velocities:
        q = _plummer_speed_fraction(rng, n)
        vesc = math.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
        vel = (q * vesc)[:, None] * _isotropic(rng, n)
    else:
        vel = np.zeros((n, 3))
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    if velocities:
        vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    pos *= a
    vel *= math.sqrt(total_mass / a)
    return pos, vel, mass


def nemo_plummer(n: int, seed: int):
    """Plummer sphere in the standard N-body units the paper's sphere generator uses.

    Standard units (G = M = 1, total energy -1/4) put the Plummer scale radius at
    3 pi / 16.  Used only to replay the paper's cumulative-error experiment
    (Sec. 3.4, Table 2), where the softening is eps^2 = 0.01.
    """
    return plummer(n, seed, a=3.0 * math.pi / 16.0)


def plummer_131072_eps(n: int = 131072) -> float:
    """Softening of the paper-scale workload: 0.1 * 4 / n^{1/3} (7.8745e-3 at n = 131072)."""
    return 0.4 / n ** (1.0 / 3.0)


def stress_system(n: int, seed: int, centre=(1000.0, 0.0, 0.0), core_frac: float = 0.1,
                  core_a: float = 1e-3):
    """Two-component precision-stress system (FP32 is not enough for its positions).

    * core: round(core_frac * n) particles, Plummer scale 1e-3 truncated at 20 scale
      radii, holding 10 % of the mass;
    * halo: the rest, Plummer scale 1 truncated at 20, holding 90 % of the mass;
    * masses drawn i.i.d. log-uniform in [1e-7, 1e-5], then each component rescaled
      to its mass fraction (total mass 1);
    * each component has its centre of mass removed in float64, then the whole
      system is moved to ``centre``; velocities are zero.

    Returns ``(pos, mass, is_core)``; the core particles come first.
    """
    rng = np.random.default_rng(seed)
    nc = int(round(core_frac * n))
    nh = n - nc
    m = np.power(10.0, rng.uniform(-7.0, -5.0, n))
    parts = []
    for cnt, scale in ((nc, core_a), (nh, 1.0)):
        r = _plummer_radii(rng, cnt, 20.0)
        parts.append(scale * r[:, None] * _isotropic(rng, cnt))
    mc, mh = m[:nc], m[nc:]
    mc *= core_frac / mc.sum()
    mh *= (1.0 - core_frac) / mh.sum()
    for p, mm in zip(parts, (mc, mh)):
        p -= (mm[:, None] * p).sum(0) / mm.sum()
    pos = np.concatenate(parts, axis=0) + np.asarray(centre, dtype=np.float64)
    is_core = np.zeros(n, dtype=bool)
    is_core[:nc] = True
    return pos, np.concatenate([mc, mh]), is_core


@dataclass
class ClusterBatch:
    """Many independent clusters stored back to back (system k owns rows offsets[k]:offsets[k+1])."""

    offsets: np.ndarray  # int64 (nsys + 1,)
    pos: np.ndarray      # float64 (total, 3)
    vel: np.ndarray      # float64 (total, 3)
    mass: np.ndarray     # float64 (total,)
    eps: np.ndarray      # float64 (nsys,)

    @property
    def nsys(self) -> int:
        return len(self.offsets) - 1

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)


def cluster_sizes(nsys: int, seed: int, nmin: int = 256, nmax: int = 16384) -> np.ndarray:
    """Cluster sizes floor(exp(U(ln nmin, ln nmax))), no rounding to tile multiples."""
    rng = np.random.default_rng(seed)
    n = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nsys))).astype(np.int64)
    return np.clip(n, nmin, nmax)


def cluster_batch(nsys: int, seed: int, nmin: int = 256, nmax: int = 16384,
                  eps: float = 0.01, velocities: bool = True) -> ClusterBatch:
    """Independent Plummer clusters (a = 1, mass 1/N_k each), one seed stream per cluster."""
    sizes = cluster_sizes(nsys, seed, nmin, nmax)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    pos = np.empty((total, 3))
    vel = np.empty((total, 3))
    mass = np.empty(total)
    for k in range(nsys):
        p, v, m = plummer(int(sizes[k]), seed=(seed * 1_000_003 + 7919 * (k + 1)) & 0x7FFFFFFF,
                          velocities=velocities)
        s, e = offsets[k], offsets[k + 1]
        pos[s:e], vel[s:e], mass[s:e] = p, v, m
    return ClusterBatch(offsets, pos, vel, mass, np.full(nsys, eps))


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """``min(k, n)`` distinct indices in [0, n), sorted, drawn with ``seed``."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def stratified_indices(mask: np.ndarray, k_each: int, seed: int) -> np.ndarray:
    """``k_each`` indices where ``mask`` holds and ``k_each`` where it does not, sorted."""
    rng = np.random.default_rng(seed)
    a = np.flatnonzero(mask)
    b = np.flatnonzero(~mask)
    sa = rng.choice(a, size=min(k_each, a.size), replace=False)
    sb = rng.choice(b, size=min(k_each, b.size), replace=False)
    return np.sort(np.concatenate([sa, sb])).astype(np.int64)


def perturbed_target(x0: np.ndarray, seed: int, scale: float = 0.01) -> np.ndarray:
    """Target positions y = x0 + scale * xi with xi ~ N(0, I) drawn with ``seed``."""
    rng = np.random.default_rng(seed)
    return x0 + scale * rng.standard_normal(x0.shape)


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload (sizes, seeds and softening of one experiment)."""

    name: str
    n: int
    eps: float
    seed: int
    dt: float = 0.0
    steps: int = 0
    description: str = ""


WORKLOADS = {
    "plummer_2048": Workload(
        "plummer_2048", 2048, 1.0 / 64.0, 1,
        description="N=2048 Plummer (a=1, M=1, equal masses, truncated at 20), v=0, eps=1/64; "
                    "one force+potential evaluation"),
    "plummer_131072": Workload(
        "plummer_131072", 131072, plummer_131072_eps(131072), 2, dt=1.0 / 256.0, steps=8,
        description="N=131072 Plummer (a=1, M=1, equal masses, truncated at 20) with "
                    "distribution-function velocities, eps=0.4/N^(1/3); force+potential and "
                    "KDK leapfrog steps dt=1/256"),
    "shard8_131072": Workload(
        "shard8_131072", 131072, plummer_131072_eps(131072), 2,
        description="one GPU's share of an 8-way i-split of the N=131072 sphere (same seed "
                    "and eps): 16384 i-particles against all 131072"),
    "active8_131072": Workload(
        "active8_131072", 131072, plummer_131072_eps(131072), 2,
        description="the N=131072 sphere of plummer_131072 (same seed and eps) with "
                    "velocities; a seeded sample of 16384 active particles against all 131072"),
    "jerk_131072": Workload(
        "jerk_131072", 131072, plummer_131072_eps(131072), 2, dt=1.0 / 256.0, steps=8,
        description="N=131072 Plummer as plummer_131072 (same seed and eps); fourth-order "
                    "Hermite steps dt=1/256, one force+jerk evaluation each"),
    "stress_1m": Workload(
        "stress_1m", 1 << 20, 1e-4, 3,
        description="N=2^20 halo + 10%-mass core of scale 1e-3 at (1000,0,0), log-uniform "
                    "masses, eps=1e-4"),
    "clusters_2048": Workload(
        "clusters_2048", 2048, 0.01, 4, dt=1.0 / 512.0, steps=16,
        description="2048 independent Plummer clusters, N_k log-uniform in [256,16384], "
                    "eps=0.01, KDK dt=1/512"),
    "adjoint_16384": Workload(
        "adjoint_16384", 16384, 0.01, 5, dt=1.0 / 256.0, steps=32,
        description="N=16384 Plummer, eps=0.01, 32 KDK steps dt=1/256; gradient of the mean "
                    "squared distance to a perturbed target"),
}
