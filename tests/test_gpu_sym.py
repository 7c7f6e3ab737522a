"""Symmetric engine (each unordered pair {i, j} evaluated once and its term added to
both particles) against the FP64 oracle.

Tolerances as for the other engines: relative RMS <= 1e-6 (compensated, FP64-reduced)
or 1e-5 (plain), and a per-particle rounding bound on every particle checked.  The
bound is that of tests/bounds.py with one change: where the j-side sum moves to the
next lane (the first i-particle of every step but the first), its term m_i r^3 d is
formed as a product and then added (a rotated sum cannot be the addend of an FMA), one
more rounding than an FMA, so an acceleration term carries up to 19 u instead of 18 u.
The j-side FP32 sums run over the 64 ipl particles of a wavefront: 16 ipl terms per
record load in a register, four loads added in the slice, so a term passes through at
most 16 ipl + 2 additions (66 for ipl = 4); the i-side blocks over 64-record chunks;
so the blocked modes' A = 127 stands; plain FP32 stays below n + 1024 additions.
Sizes cover one block row (only the diagonal), ragged rows and tiles, several
segments per row, and the N = 131072 sphere on sampled particles.
"""
import numpy as np
import pytest
import torch

import bounds
import oracle
from paper_astro_ph_0703100_amd import _lib, api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"comp": 1e-6, "fp64red": 1e-6, "plain": 1e-5}
U = bounds.U
C_ACC_SYM = bounds.C_ACC + 1.0

SHAPES = [(1, 64), (1, 128), (2, 64), (2, 128), (4, 64), (4, 128)]


def to_dev(pos, mass):
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    return (torch.from_numpy(p32).to(DEV), torch.from_numpy(m32).to(DEV),
            p32.T.astype(np.float64), m32.astype(np.float64))


def check(acc, pot, ra, rp, x64, m64, eps, precision, idx=None):
    n = x64.shape[0]
    idx = np.arange(n) if idx is None else idx
    absa, absp = oracle.force_abs_sampled(x64, m64, eps, idx)
    a = bounds.adds(precision, n)
    ratio_a = np.abs(acc - ra) / (U * np.maximum(absa, 1e-300))
    assert ratio_a.max() <= C_ACC_SYM + a, (precision, float(ratio_a.max()))
    wp = 0.0
    if pot is not None:
        ratio_p = np.abs(pot - rp) / (U * np.maximum(absp, 1e-300))
        assert ratio_p.max() <= bounds.C_POT + a, (precision, float(ratio_p.max()))
        wp = float(ratio_p.max())
    return float(ratio_a.max()), wp


def sym_force(p, m, eps, **kw):
    acc, pot = api.force(p, m, eps, symmetric=2, **kw)
    torch.cuda.synchronize()
    return acc, pot


@pytest.mark.parametrize("ipl,jt", SHAPES)
def test_sym_shapes_match_oracle(ipl, jt):
    n = 3001
    pos, _, mass = ics.plummer(n, seed=700 + jt, velocities=False)
    mass = mass * np.random.default_rng(ipl + jt).uniform(0.5, 1.5, n)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    for precision in ("comp", "fp64red", "plain"):
        acc, pot = sym_force(p, m, eps, precision=precision, ipl=ipl, jtile=jt)
        acc2, pot2 = sym_force(p, m, eps, precision=precision, ipl=ipl, jtile=jt)
        assert torch.equal(acc, acc2) and torch.equal(pot, pot2)  # reproducible
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
        wa, wp = check(acc, pot, ra, rp, x64, m64, eps, precision)
        print(ipl, jt, precision, "acc", ea, "pot", ep, "bound ratios %.1f %.1f" % (wa, wp))
        assert ea["rel_rms"] <= TOL[precision], (precision, ea)
        assert ep["rel_rms"] <= TOL[precision], (precision, ep)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 2048, 4097])
def test_sym_ragged_sizes(n):
    pos, _, mass = ics.plummer(n, seed=1900 + n, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.02
    ra, rp = oracle.force_all(x64, m64, eps)
    for ipl, jt in [(1, 128), (2, 64), (4, 64), (4, 128)]:
        acc, pot = sym_force(p, m, eps, ipl=ipl, jtile=jt)
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        if n == 1:
            assert np.all(acc == 0) and np.all(pot == 0)
            continue
        assert rel_errors(acc, ra)["rel_rms"] <= 1e-6
        check(acc, pot, ra, rp, x64, m64, eps, "comp")


@pytest.mark.parametrize("nseg", [1, 2, 7, 1000])
def test_sym_segments(nseg):
    """Work items of 1 to all j-tiles of a row (nseg larger than a row's tiles is capped):
    every pair counted once whatever the split."""
    n = 6000
    pos, _, mass = ics.plummer(n, seed=31 + nseg, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    for ipl, jt in [(1, 64), (2, 128), (4, 64)]:
        acc, pot = sym_force(p, m, eps, ipl=ipl, jtile=jt, nseg=nseg)
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        assert rel_errors(acc, ra)["rel_rms"] <= 1e-6
        assert rel_errors(pot, rp)["rel_rms"] <= 1e-6
        check(acc, pot, ra, rp, x64, m64, eps, "comp")


def test_sym_momentum_and_grid_agreement():
    """Each pair's two terms come from the same separation and 1/s: the mass-weighted
    sum of the accelerations cancels to the accumulation rounding, and the engine agrees
    with the grid engine to the pair rounding."""
    n = 5000
    pos, _, mass = ics.plummer(n, seed=12, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    acc, _ = sym_force(p, m, eps)
    accg, _ = api.force(p, m, eps, symmetric=1, jlanes=1)
    torch.cuda.synchronize()
    a, g = acc.cpu().numpy().T, accg.cpu().numpy().T
    absa, _ = oracle.force_abs_sampled(x64, m64, eps, np.arange(n))
    f = (m64[:, None] * a).sum(axis=0)
    scale = (m64[:, None] * absa).sum(axis=0)
    print("momentum", f / scale)
    assert np.all(np.abs(f) <= 1e-6 * scale)
    assert rel_errors(a, g)["rel_rms"] <= 1e-6


def test_sym_self_potential_and_no_potential():
    n = 1777
    pos, _, mass = ics.plummer(n, seed=8, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    acc, pot = api.force(p, m, eps, self_pot=True, symmetric=2, jtile=128)
    acc0, pot0 = api.force(p, m, eps, with_pot=False, symmetric=2, jtile=128)
    acc1, _ = api.force(p, m, eps, symmetric=2, jtile=128)
    torch.cuda.synchronize()
    assert pot0 is None
    assert torch.equal(acc0, acc1)  # the potential-free kernel sums the same terms
    pot = pot.cpu().numpy()
    assert rel_errors(pot, rp - m64 / np.float64(np.float32(eps)))["rel_rms"] <= 1e-6


def test_sym_coincident_particles():
    """Particles at the same place in different block rows: s = eps, finite terms."""
    n = 1500
    pos, _, mass = ics.plummer(n, seed=3, velocities=False)
    pos[1200] = pos[5]
    pos[700] = pos[5]
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    acc, pot = sym_force(p, m, eps, jtile=64)
    acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    check(acc, pot, ra, rp, x64, m64, eps, "comp")


def test_sym_force_f64_system_centre_and_leapfrog():
    """FP64 positions with the system centre, and two KDK steps, on the symmetric engine:
    the force within tolerance of the oracle, the trajectory next to the grid engine's."""
    n = 4096
    pos, vel, mass = ics.plummer(n, seed=56)
    pos = pos + 100.0
    m32 = mass.astype(np.float32)
    m64 = m32.astype(np.float64)
    m = torch.from_numpy(m32).to(DEV)
    eps, dt = 0.01, 1.0 / 256
    p64 = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    acc, pot = api.force_f64(p64, m, eps, symmetric=2)
    torch.cuda.synchronize()
    ra, rp = oracle.force_all(pos, m64, eps)
    assert rel_errors(acc.cpu().numpy().T, ra)["rel_rms"] <= 1e-6
    assert rel_errors(pot.cpu().numpy(), rp)["rel_rms"] <= 1e-6
    out = {}
    for name, kw in (("sym", dict(symmetric=2)), ("grid", dict(symmetric=1, jlanes=1))):
        x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
        v = torch.from_numpy(np.ascontiguousarray(vel.T)).to(DEV)
        a, pt, _ = api.leapfrog(x, v, m, eps, dt, 2, with_pot=True, **kw)
        torch.cuda.synchronize()
        out[name] = (x.cpu().numpy().T, a.cpu().numpy().T, pt.cpu().numpy())
    xs, a, pt = out["sym"]
    ra, rp = oracle.force_all(xs, m64, eps)
    assert rel_errors(a, ra)["rel_rms"] <= 1e-6
    assert rel_errors(pt, rp)["rel_rms"] <= 1e-6
    assert np.abs(out["sym"][0] - out["grid"][0]).max() < 1e-9


def test_sym_leapfrog_graph_replays_match_eager_steps():
    """Captured KDK steps on the symmetric engine (the graph owns its scratch): every
    replay, with eager work between them, gives bitwise the eager steps' state."""
    n, steps, dt, eps = 3000, 3, 1.0 / 256, 0.01
    pos, vel, mass = ics.plummer(n, seed=66)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    shape = dict(ipl=1, jtile=128, symmetric=2)

    def fresh():
        return (torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV),
                torch.from_numpy(np.ascontiguousarray(vel.T)).to(DEV))
    xe, ve = fresh()
    ae, _, _ = api.leapfrog(xe, ve, m, eps, dt, 0, **shape)
    xg, vg = xe.clone(), ve.clone()
    ag = ae.clone()
    g = api.LeapfrogGraph(xg, vg, m, eps, dt, steps, ag, **shape)
    for _ in range(3):
        api.leapfrog(xe, ve, m, eps, dt, steps, acc=ae, init=False, **shape)
        g.launch()
        api.force(torch.zeros((3, 8), device=DEV), torch.ones(8, device=DEV), 0.1)  # eager work
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(vg, ve) and torch.equal(ag, ae)
    g.close()


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_sym_plummer_131072_sampled(precision):
    """The N = 131072 sphere on the symmetric engine (its default shape for this size):
    full sum on the GPU, oracle on 2048 seeded sample particles, bound on each."""
    w = ics.WORKLOADS["plummer_131072"]
    pos, _, mass = ics.plummer(w.n, seed=w.seed)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = float(np.float32(w.eps))
    acc, pot = sym_force(p, m, eps, precision=precision)
    acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
    idx = ics.sample_indices(w.n, 2048, seed=w.seed + 2000)
    ra, rp = oracle.force_sampled(x64, m64, eps, idx)
    ea, ep = rel_errors(acc[idx], ra), rel_errors(pot[idx], rp)
    wa, wp = check(acc[idx], pot[idx], ra, rp, x64, m64, eps, precision, idx)
    print(precision, "acc", ea, "pot", ep, "bound ratios %.1f %.1f" % (wa, wp))
    assert ea["rel_rms"] <= TOL[precision] and ep["rel_rms"] <= TOL[precision]


def test_sym_rejected_where_not_built():
    n = 1000
    pos, _, mass = ics.plummer(n, seed=5, velocities=False)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    with pytest.raises(_lib.NBodyError) as e:
        api.force_ij(p, p, m, 0.01, symmetric=2)
    assert e.value.status == _lib.NBODY_EUNSUPPORTED
    with pytest.raises(_lib.NBodyError) as e:
        api.force(p, m, 0.01, symmetric=2, jtile=512)
    assert e.value.status == _lib.NBODY_EINVAL
