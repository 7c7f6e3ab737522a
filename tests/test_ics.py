"""Checks of the seeded synthetic workloads (shape, determinism and physical sanity)."""
import math

import numpy as np

import oracle
from paper_astro_ph_0703100_amd import ics


def test_plummer_is_deterministic_and_centred():
    a = ics.plummer(1000, seed=5)
    b = ics.plummer(1000, seed=5)
    c = ics.plummer(1000, seed=6)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    assert not np.array_equal(a[0], c[0])
    pos, vel, m = a
    assert pos.shape == (1000, 3) and vel.shape == (1000, 3) and m.shape == (1000,)
    assert abs(m.sum() - 1.0) < 1e-14
    assert np.abs((m[:, None] * pos).sum(0)).max() < 1e-14
    assert np.abs((m[:, None] * vel).sum(0)).max() < 1e-14
    assert np.linalg.norm(pos, axis=1).max() <= 20.0 + 1.0


def test_plummer_mass_profile():
    # Fraction inside r = 1 of a Plummer sphere truncated at 20: M(1)/M(20).
    n = 32768
    pos, _, _ = ics.plummer(n, seed=7, velocities=False)
    r = np.linalg.norm(pos, axis=1)
    p = (1 / 2 ** 1.5) / (20 ** 3 / (1 + 400) ** 1.5)
    sigma = math.sqrt(p * (1 - p) / n)
    assert abs((r < 1).mean() - p) < 4 * sigma
    half = np.median(r)
    # Half-mass radius of the untruncated model is (2^{2/3} - 1)^{-1/2} = 1.305.
    assert abs(half - 1.305) < 0.05


def test_plummer_virial_equilibrium():
    # 2T / |W| = 1 for the distribution-function velocities (softening and
    # truncation move it by a few per cent at most).
    x, v, m = ics.plummer(4096, seed=8)
    _, pot = oracle.force_all(x, m, 1e-3)
    t = 0.5 * np.sum(m * np.sum(v * v, axis=1))
    w = 0.5 * np.sum(m * pot)
    assert abs(2 * t / abs(w) - 1.0) < 0.06


def test_nemo_units_energy():
    # Standard N-body units: total energy -1/4 (to discreteness noise).
    x, v, m = ics.nemo_plummer(4096, seed=9)
    e = oracle.energy(x, v, m, 1e-3)
    assert abs(e + 0.25) < 0.02


def test_stress_system():
    n = 20000
    pos, m, core = ics.stress_system(n, seed=3)
    assert core.sum() == 2000
    assert abs(m[core].sum() - 0.1) < 1e-13 and abs(m.sum() - 1.0) < 1e-13
    assert m.min() > 0
    com_core = (m[core, None] * pos[core]).sum(0) / m[core].sum()
    np.testing.assert_allclose(com_core, [1000.0, 0, 0], atol=1e-9)
    assert np.linalg.norm(pos[core] - [1000.0, 0, 0], axis=1).max() < 2.1e-2


def test_cluster_batch_sizes():
    sizes = ics.cluster_sizes(2048, seed=4)
    assert sizes.min() >= 256 and sizes.max() <= 16384
    # Log-uniform: mean (16384 - 256) / ln 64 = 3878, sum of squares about 6.6e10.
    assert abs(sizes.mean() / 3878.0 - 1) < 0.06
    assert abs((sizes.astype(float) ** 2).sum() / 6.6e10 - 1) < 0.1
    b = ics.cluster_batch(6, seed=4)
    assert b.offsets[0] == 0 and b.offsets[-1] == b.pos.shape[0]
    for k in range(6):
        s, e = b.offsets[k], b.offsets[k + 1]
        assert abs(b.mass[s:e].sum() - 1.0) < 1e-12


def test_sampling_helpers():
    idx = ics.sample_indices(100, 10, seed=1)
    assert idx.size == 10 and np.all(np.diff(idx) > 0)
    np.testing.assert_array_equal(idx, ics.sample_indices(100, 10, seed=1))
    assert ics.sample_indices(5, 10, seed=1).size == 5
    mask = np.zeros(50, dtype=bool)
    mask[:7] = True
    s = ics.stratified_indices(mask, 5, seed=2)
    assert mask[s].sum() == 5 and (~mask[s]).sum() == 5
    assert abs(ics.plummer_131072_eps() - 7.8745e-3) < 1e-6
