"""GPU parity of the separate i-/j-set force path (nbody_force_ij) against the oracle.

The i-set and the j-set are different particles (or an i-range of one system against
all of it); every pair counts, and the softening is uniform or given per i-particle.
Tolerances as for the single-set path: compensated and FP64-reduced relative RMS
<= 1e-6, plain FP32 <= 1e-5, and (uniform softening) the per-particle rounding bound
of tests/bounds.py on every component.
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


def dev_soa(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a.T.astype(dtype))).to(DEV)


def run_ij(xi, xj, mj, eps=0.0, eps_i=None, **kw):
    acc, pot = api.force_ij(dev_soa(xi), dev_soa(xj), torch.from_numpy(mj.astype(np.float32)).to(DEV),
                            eps, eps_i=None if eps_i is None else
                            torch.from_numpy(eps_i.astype(np.float32)).to(DEV), **kw)
    torch.cuda.synchronize()
    return acc.cpu().numpy().T, pot.cpu().numpy() if pot is not None else None


def as32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
@pytest.mark.parametrize("ni,nj", [(3001, 5003), (257, 20000), (9000, 300), (1, 1), (5, 64)])
def test_separate_sets_uniform_eps(precision, ni, nj):
    xi, _, _ = ics.plummer(ni, seed=200 + ni, velocities=False)
    xj, _, mj = ics.plummer(nj, seed=300 + nj, velocities=False)
    xi = xi * 1.3 + 0.05  # the two sets are different particles
    mj = mj * np.random.default_rng(nj).uniform(0.5, 1.5, nj)
    eps = float(np.float32(0.02))
    acc, pot = run_ij(xi, xj, mj, eps, precision=precision)
    ra, rp = oracle.force_ij(as32(xj), as32(mj), as32(xi), eps)
    ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
    absa, absp = oracle.force_abs(as32(xj), as32(mj), as32(xi), eps)
    wa = bounds.check_acc(acc, ra, absa, precision, nj)
    wp = bounds.check_pot(pot, rp, absp, precision, nj)
    print(precision, ni, nj, "acc", ea, "pot", ep, "bound ratios %.2f %.2f" % (wa, wp))
    assert ea["rel_rms"] <= TOL[precision], ea
    assert ep["rel_rms"] <= TOL[precision], ep


@pytest.mark.parametrize("precision", ["comp", "plain"])
def test_per_i_softening_including_zero(precision):
    ni, nj = 4100, 3333  # ragged i- and j-tails: padding records are used
    rng = np.random.default_rng(41)
    xi, _, _ = ics.plummer(ni, seed=41, velocities=False)
    xj, _, mj = ics.plummer(nj, seed=42, velocities=False)
    eps_i = rng.uniform(0.0, 0.05, ni).astype(np.float32)
    eps_i[::7] = 0.0  # unsoftened i's: no j sits exactly on an i
    acc, pot = run_ij(xi, xj, mj, eps=0.5, eps_i=eps_i, precision=precision)
    ra, rp = oracle.force_ij(as32(xj), as32(mj), as32(xi), None, eps_i=eps_i.astype(np.float64))
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
    print(precision, "acc", ea, "pot", ep)
    # Unsoftened close pairs make single terms large; the bound is per-term rounding.
    assert ea["rel_rms"] <= 10 * TOL[precision], ea
    assert ep["rel_rms"] <= TOL[precision], ep


def test_eps_zero_uniform_with_padding():
    # eps = 0 and an i-particle at the origin: padding j-records (far away, massless)
    # must add exactly nothing, so the result is finite and matches the oracle.
    xi = np.array([[0.0, 0.0, 0.0], [0.5, -0.25, 0.125], [3.0, 1.0, -2.0]])
    xj, _, mj = ics.plummer(77, seed=77, velocities=False)
    xj = xj + 0.01  # keep every j off the i's
    acc, pot = run_ij(xi, xj, mj, eps=0.0, precision="comp")
    ra, rp = oracle.force_ij(as32(xj), as32(mj), as32(xi), 0.0)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    assert rel_errors(acc, ra)["e_max"] <= 1e-5
    assert rel_errors(pot, rp)["e_max"] <= 1e-6


def test_empty_j_set_writes_zeros_and_empty_i_set_is_a_no_op():
    xi = dev_soa(np.ones((5, 3)))
    xj = torch.empty((3, 0), dtype=torch.float32, device=DEV)
    mj = torch.empty(0, dtype=torch.float32, device=DEV)
    acc = torch.full((3, 5), 7.0, dtype=torch.float64, device=DEV)
    pot = torch.full((5,), 7.0, dtype=torch.float64, device=DEV)
    api.force_ij(xi, xj, mj, 0.1, out=(acc, pot))
    torch.cuda.synchronize()
    assert torch.all(acc == 0) and torch.all(pot == 0)
    xe = torch.empty((3, 0), dtype=torch.float32, device=DEV)
    a0, p0 = api.force_ij(xe, xi, torch.ones(5, dtype=torch.float32, device=DEV), 0.1)
    torch.cuda.synchronize()
    assert a0.shape == (3, 0) and p0.shape == (0,)


@pytest.mark.parametrize("precision", ["comp", "fp64red"])
def test_i_range_shard_matches_the_whole_system(precision):
    # One GPU's share of a system split by i: its i-range against all j's.  Accelerations
    # equal the single-set path's on that range; the potential differs by the self term
    # -m_i/eps, which a separate i-set includes (its own j copy is just another j).
    n = 20000
    pos, _, mass = ics.plummer(n, seed=55, velocities=False)
    p = dev_soa(pos)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    eps = float(np.float32(0.01))
    acc_all, pot_all = api.force(p, m, eps, precision=precision)
    for i0, i1 in [(0, 2500), (2500, 10001), (10001, 20000)]:
        pi = p[:, i0:i1].contiguous()
        acc, pot = api.force_ij(pi, p, m, eps, precision=precision)
        torch.cuda.synchronize()
        a_ref = acc_all[:, i0:i1].cpu().numpy().T
        e = rel_errors(acc.cpu().numpy().T, a_ref)
        assert e["rel_rms"] <= 2e-7, e
        m64 = mass.astype(np.float32).astype(np.float64)[i0:i1]
        self_term = m64 * (1.0 / np.sqrt(np.float64(np.float32(eps) * np.float32(eps))))
        p_ref = pot_all[i0:i1].cpu().numpy() - self_term
        assert rel_errors(pot.cpu().numpy(), p_ref)["rel_rms"] <= 1e-6


def test_full_size_shard_sampled():
    # The i-sharded shape at paper scale: 1/8 of N = 131072 against all of it, in the
    # tuned launch shape; 512 sampled i's against the oracle.
    w = ics.WORKLOADS["plummer_131072"]
    pos, _, mass = ics.plummer(w.n, seed=w.seed, velocities=False)
    eps = float(np.float32(w.eps))
    ni = w.n // 8
    acc, pot = run_ij(pos[:ni], pos, mass, eps, precision="comp")
    idx = ics.sample_indices(ni, 512, seed=77)
    ra, rp = oracle.force_ij(as32(pos), as32(mass), as32(pos[idx]), eps)
    ea, ep = rel_errors(acc[idx], ra), rel_errors(pot[idx], rp)
    absa, absp = oracle.force_abs(as32(pos), as32(mass), as32(pos[idx]), eps)
    wa = bounds.check_acc(acc[idx], ra, absa, "comp", w.n)
    wp = bounds.check_pot(pot[idx], rp, absp, "comp", w.n)
    print("shard acc", ea, "pot", ep, "bound ratios %.2f %.2f" % (wa, wp))
    assert ea["rel_rms"] <= 1e-6, ea
    assert ep["rel_rms"] <= 1e-6, ep


def test_launch_shapes_and_workspace():
    ni, nj = 2000, 7000
    xi, _, _ = ics.plummer(ni, seed=61, velocities=False)
    xj, _, mj = ics.plummer(nj, seed=62, velocities=False)
    ra, _ = oracle.force_ij(as32(xj), as32(mj), as32(xi), 0.03)
    for ipl, jt, nseg in [(1, 64, 1), (2, 512, 5), (4, 128, 0), (8, 256, 13)]:
        o = dict(ipl=ipl, jtile=jt, nseg=nseg)
        need = _lib.nbody_workspace_size_ij(ni, nj, api.make_opts(**o))
        assert need > 0
        ws = torch.empty(need // 4, dtype=torch.float32, device=DEV)
        acc, _ = run_ij(xi, xj, mj, 0.03, precision="comp", workspace=ws, **o)
        assert rel_errors(acc, ra)["rel_rms"] <= 1e-6, o
