"""GPU parity of the force/potential path against the FP64 oracle.

Both sides see the same seeded particles: the GPU the FP32 (or FP64) arrays, the
oracle the same values promoted to FP64, so the comparison measures the GPU's
arithmetic only.  Tolerances:
  * compensated and FP64-reduced accumulation: relative RMS acceleration error
    <= 1e-6 (and the same for the potential);
  * plain FP32 accumulation is reported and only checked against a loose bound
    (its error grows with the number of terms per accumulator);
  * every particle: the per-component rounding bound of tests/bounds.py on the
    acceleration and the potential (error <= (C + A) u times the sum of the terms'
    magnitudes), so an error confined to a few particles cannot hide in an RMS.
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


def to_dev(pos, mass):
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    return (torch.from_numpy(p32).to(DEV), torch.from_numpy(m32).to(DEV),
            p32.T.astype(np.float64), m32.astype(np.float64))


def check_bounds(acc, pot, ra, rp, x64, m64, eps, precision, idx=None):
    """Per-particle bounds of tests/bounds.py on the listed particles (all if None)."""
    n = x64.shape[0]
    idx = np.arange(n) if idx is None else idx
    absa, absp = oracle.force_abs_sampled(x64, m64, eps, idx)
    wa = bounds.check_acc(acc, ra, absa, precision, n)
    wp = bounds.check_pot(pot, rp, absp, precision, n) if pot is not None else 0.0
    return wa, wp


def gpu_force(p, m, eps, **kw):
    acc, pot = api.force(p, m, eps, **kw)
    torch.cuda.synchronize()
    return acc.cpu().numpy().T, pot.cpu().numpy() if pot is not None else None


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_plummer_2048_full_parity(precision):
    w = ics.WORKLOADS["plummer_2048"]
    pos, _, mass = ics.plummer(w.n, seed=w.seed, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = float(np.float32(w.eps))
    acc, pot = gpu_force(p, m, eps, precision=precision)
    ra, rp = oracle.force_all(x64, m64, eps)
    ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
    wa, wp = check_bounds(acc, pot, ra, rp, x64, m64, eps, precision)
    print(precision, "acc", ea, "pot", ep, "worst err / (u sum|t|): acc %.2f pot %.2f" % (wa, wp))
    assert ea["rel_rms"] <= TOL[precision], ea
    assert ep["rel_rms"] <= TOL[precision], ep


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 257, 1000, 1023, 1025, 2049, 3001])
def test_ragged_sizes(n):
    pos, _, mass = ics.plummer(n, seed=100 + n, velocities=False)
    mass = mass * np.random.default_rng(n).uniform(0.5, 1.5, n)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.03
    ra, rp = oracle.force_all(x64, m64, eps)
    for precision in ("comp", "fp64red", "plain"):
        acc, pot = gpu_force(p, m, eps, precision=precision)
        if n == 1:
            assert np.all(acc == 0) and np.all(pot == 0)
            continue
        ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
        assert ea["rel_rms"] <= TOL[precision], (precision, ea)
        check_bounds(acc, pot, ra, rp, x64, m64, eps, precision)


@pytest.mark.parametrize("ipl,jtile,nseg", [(1, 64, 1), (1, 512, 3), (2, 128, 7), (4, 256, 2),
                                             (8, 64, 5), (8, 512, 1), (4, 128, 40)])
def test_launch_shapes_agree_with_oracle(ipl, jtile, nseg):
    n = 5000
    pos, _, mass = ics.plummer(n, seed=7, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    ra, rp = oracle.force_all(x64, m64, 0.01)
    for precision in ("comp", "plain"):
        acc, pot = gpu_force(p, m, 0.01, precision=precision, ipl=ipl, jtile=jtile, nseg=nseg)
        ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
        assert ea["rel_rms"] <= TOL[precision] and ep["rel_rms"] <= TOL[precision], (precision, ea, ep)
        check_bounds(acc, pot, ra, rp, x64, m64, 0.01, precision)


def test_without_potential_and_with_self_term():
    n = 777
    pos, _, mass = ics.plummer(n, seed=8, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = float(np.float32(0.02))
    acc_np, _ = gpu_force(p, m, eps, with_pot=False)
    acc, pot = gpu_force(p, m, eps)
    np.testing.assert_array_equal(acc_np, acc)
    acc_self, pot_self = gpu_force(p, m, eps, self_pot=True)
    # Including the self term subtracts m_i / eps, formed in FP64, from each potential;
    # the sums themselves are the same bits.
    np.testing.assert_array_equal(acc_self, acc)
    np.testing.assert_array_equal(pot_self, pot - m64 / eps)


def test_zero_and_one_particle():
    e = torch.empty(0, device=DEV)
    _lib.nbody_force(0, e.data_ptr(), e.data_ptr(), 0.1, e.data_ptr(), None, None)
    p = torch.tensor([[1.0], [2.0], [3.0]], dtype=torch.float32, device=DEV)
    m = torch.tensor([2.0], dtype=torch.float32, device=DEV)
    acc, pot = gpu_force(p, m, 0.1)
    assert np.all(acc == 0) and np.all(pot == 0)


def test_coincident_particles():
    pos = np.array([[0.25, -0.5, 1.0]] * 3)
    mass = np.array([1.0, 2.0, 4.0])
    p, m, _, _ = to_dev(pos, mass)
    acc, pot = gpu_force(p, m, 0.25)
    assert np.all(acc == 0)
    np.testing.assert_allclose(pot, [-24.0, -20.0, -12.0], rtol=1e-6)


def test_deterministic_reruns():
    n = 20000
    pos, _, mass = ics.plummer(n, seed=9, velocities=False)
    p, m, _, _ = to_dev(pos, mass)
    a1, p1 = gpu_force(p, m, 0.01)
    a2, p2 = gpu_force(p, m, 0.01)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(p1, p2)


def test_power_of_two_scaling():
    # x -> 4x, eps -> 4 eps scales a by 1/16 and phi by 1/4 (a change of exponent only).
    n = 3000
    pos, _, mass = ics.plummer(n, seed=10, velocities=False)
    p, m, _, _ = to_dev(pos, mass)
    a1, p1 = gpu_force(p, m, 0.01)
    a4, p4 = gpu_force(p * 4.0, m, 0.04)
    np.testing.assert_allclose(a4, a1 / 16.0, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(p4, p1 / 4.0, rtol=1e-6)


def test_momentum_conservation():
    n = 8192
    pos, _, mass = ics.plummer(n, seed=11, velocities=False)
    p, m, _, m64 = to_dev(pos, mass)
    acc, _ = gpu_force(p, m, 0.01)
    resid = np.abs((m64[:, None] * acc).sum(0))
    scale = (m64[:, None] * np.abs(acc)).sum(0)
    assert np.all(resid < 1e-7 * scale), resid / scale


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_plummer_131072_sampled_parity(precision):
    """Paper-scale sphere: full GPU sum, oracle on 4096 seeded sample particles."""
    w = ics.WORKLOADS["plummer_131072"]
    pos, _, mass = ics.plummer(w.n, seed=w.seed)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = float(np.float32(w.eps))
    acc, pot = gpu_force(p, m, eps, precision=precision)
    idx = ics.sample_indices(w.n, 4096, seed=w.seed + 1000)
    ra, rp = oracle.force_sampled(x64, m64, eps, idx)
    ea, ep = rel_errors(acc[idx], ra), rel_errors(pot[idx], rp)
    wa, wp = check_bounds(acc[idx], pot[idx], ra, rp, x64, m64, eps, precision, idx)
    print(precision, "acc", ea, "pot", ep, "worst err / (u sum|t|): acc %.2f pot %.2f" % (wa, wp))
    assert ea["rel_rms"] <= TOL[precision], ea
    assert ep["rel_rms"] <= TOL[precision], ep


def test_force_f64_centres():
    """FP64 positions far from the origin: a system centre restores FP32 accuracy."""
    n = 20000
    pos, mass, core = ics.stress_system(n, seed=3)
    p64 = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    m64 = mass.astype(np.float32).astype(np.float64)
    eps = float(np.float32(1e-4))
    idx = ics.stratified_indices(core, 256, seed=1003)
    ra, rp = oracle.force_sampled(pos, m64, eps, idx)
    acc, pot = api.force_f64(p64, m, eps, centre="system")
    torch.cuda.synchronize()
    e_sys = rel_errors(acc.cpu().numpy().T[idx], ra)
    acc0, _ = api.force_f64(p64, m, eps, centre="none")
    torch.cuda.synchronize()
    e_none = rel_errors(acc0.cpu().numpy().T[idx], ra)
    print("centre system", e_sys, "none", e_none)
    assert e_sys["rel_rms"] < 1e-5
    assert e_none["rel_rms"] > 10 * e_sys["rel_rms"]
