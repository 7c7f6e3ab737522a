"""GPU parity of the separate-set force-jerk-potential path (nbody_force_jerk_ij).

The i-set and the j-set are different particles (for example the active particles of
a Hermite code with individual steps against all of them); every pair counts.
Acceleration and potential: relative RMS <= 1e-6 compensated / FP64-reduced, 1e-5
plain.  The jerk is bounded per particle by the arithmetic, as for nbody_force_jerk:
|Delta jerk_i| <= (74 + A - 1) u sum_j B_ij with B_ij = m_j (|w| / s^3 + 3 |d.w| |d| /
s^5), A = 128 FP32 additions per compensation block (plain FP32: the segment and its
segment sum, < n_j + 1024).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import _lib, api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U = 2.0 ** -24
TOL = {"comp": 1e-6, "fp64red": 1e-6, "plain": 1e-5}


def as32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def soa(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32).T)).to(DEV)


def run(xi, vi, xj, vj, mj, eps, **kw):
    acc, jerk, pot = api.force_jerk_ij(soa(xi), soa(vi), soa(xj), soa(vj),
                                       torch.from_numpy(mj.astype(np.float32)).to(DEV), eps, **kw)
    torch.cuda.synchronize()
    return acc.cpu().numpy().T, jerk.cpu().numpy().T, pot.cpu().numpy() if pot is not None else None


def jerk_scale(xi, vi, xj, vj, mj, eps):
    e2 = eps * eps
    out = np.empty(len(xi))
    for i in range(len(xi)):
        d, w = xj - xi[i], vj - vi[i]
        s2 = (d * d).sum(1) + e2
        dn = np.sqrt((d * d).sum(1))
        out[i] = (mj * (np.sqrt((w * w).sum(1)) / s2 ** 1.5
                        + 3 * np.abs((d * w).sum(1)) * dn / s2 ** 2.5)).sum()
    return out


def check(got, ref, scale, precision, nj):
    acc, jerk, pot = got
    ra, rj, rp = ref
    assert rel_errors(acc, ra)["rel_rms"] <= TOL[precision]
    if pot is not None:
        assert rel_errors(pot, rp)["rel_rms"] <= TOL[precision]
    c = 74.0 + (nj + 1024 if precision == "plain" else 127)
    err = np.sqrt(((jerk - rj) ** 2).sum(1))
    assert np.all(err <= c * U * scale), (precision, float((err / (U * scale + 1e-300)).max()))


def two_sets(ni, nj, seed, offset=0.05):
    xi, vi, _ = ics.plummer(ni, seed=seed)
    xj, vj, mj = ics.plummer(nj, seed=seed + 1)
    mj = mj * np.random.default_rng(seed + 2).uniform(0.5, 1.5, nj)
    return as32(xi * 1.3 + offset), as32(vi), as32(xj), as32(vj), as32(mj)


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
@pytest.mark.parametrize("ni,nj", [(3001, 5003), (257, 20000), (9000, 300), (1, 1), (5, 64)])
def test_separate_sets(precision, ni, nj):
    xi, vi, xj, vj, mj = two_sets(ni, nj, 500 + ni)
    eps = float(np.float32(0.02))
    got = run(xi, vi, xj, vj, mj, eps, precision=precision)
    ref = oracle.force_jerk_ij(xj, vj, mj, xi, vi, eps)
    check(got, ref, jerk_scale(xi, vi, xj, vj, mj, eps), precision, nj)


@pytest.mark.parametrize("precision", ["comp", "plain"])
def test_zero_softening_between_separated_sets(precision):
    # eps = 0 is allowed for separate sets; the sets sit 4 units apart so no pair is
    # close, and the ragged tails exercise the far, massless padding records.
    xi, vi, xj, vj, mj = two_sets(777, 3001, 61, offset=4.0)
    got = run(xi, vi, xj, vj, mj, 0.0, precision=precision)
    assert all(np.all(np.isfinite(g)) for g in got)
    ref = oracle.force_jerk_ij(xj, vj, mj, xi, vi, 0.0)
    check(got, ref, jerk_scale(xi, vi, xj, vj, mj, 0.0), precision, 3001)


@pytest.mark.parametrize("ipl,jtile,nseg", [(1, 64, 1), (2, 128, 7), (4, 256, 3), (8, 512, 2),
                                             (1, 128, 200)])
def test_launch_shapes(ipl, jtile, nseg):
    xi, vi, xj, vj, mj = two_sets(2500, 4100, 71)
    eps = float(np.float32(0.03))
    got = run(xi, vi, xj, vj, mj, eps, ipl=ipl, jtile=jtile, nseg=nseg)
    ref = oracle.force_jerk_ij(xj, vj, mj, xi, vi, eps)
    check(got, ref, jerk_scale(xi, vi, xj, vj, mj, eps), "comp", 4100)


def test_one_set_gives_the_single_set_sums():
    # i-set = j-set at the same launch shape: the j == i pair adds exactly zero to a and
    # the jerk in both paths and the padding adds exactly zero, so a and the jerk are
    # bitwise those of nbody_force_jerk; phi differs by the self term only.
    x, v, m = ics.plummer(3000, seed=81)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(0.02))
    shape = dict(ipl=1, jtile=128, nseg=5)
    a1, j1, p1 = api.force_jerk(soa(x), soa(v), torch.from_numpy(m.astype(np.float32)).to(DEV),
                                eps, **shape)
    a2, j2, p2 = api.force_jerk_ij(soa(x), soa(v), soa(x), soa(v),
                                   torch.from_numpy(m.astype(np.float32)).to(DEV), eps, **shape)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(j1, j2)
    self_term = torch.from_numpy(m / eps).to(DEV)
    assert torch.allclose(p2, p1 - self_term, rtol=1e-6, atol=0)


def test_active_subset_of_the_paper_sphere():
    # 4096 'active' particles of the N = 131072 sphere against all of it, checked on
    # every active particle.
    w = ics.WORKLOADS["jerk_131072"]
    x, v, m = ics.plummer(w.n, seed=w.seed)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(w.eps))
    idx = ics.sample_indices(w.n, 4096, seed=91)
    got = run(x[idx], v[idx], x, v, m, eps)
    ra, rj, rp = oracle.force_jerk_ij(x, v, m, x[idx], v[idx], eps)
    # The i-set is part of the j-set: the oracle sums the j == i pair too (-m_i/eps in phi).
    assert rel_errors(got[0], ra)["rel_rms"] <= 1e-6
    assert rel_errors(got[2], rp)["rel_rms"] <= 1e-6
    assert rel_errors(got[1], rj)["normwise"] <= 1e-5


def test_empty_sets_and_workspace():
    xi, vi, xj, vj, mj = two_sets(100, 200, 95)
    # nj = 0: zeros.
    acc, jerk, pot = api.force_jerk_ij(soa(xi), soa(vi), soa(xj[:0]), soa(vj[:0]),
                                       torch.zeros(0, dtype=torch.float32, device=DEV), 0.1)
    torch.cuda.synchronize()
    assert not acc.any() and not jerk.any() and not pot.any()
    # A caller workspace of the reported size gives the same bits as the library's own.
    opts = api.make_opts()
    need = _lib.nbody_workspace_size_jerk_ij(100, 200, opts)
    assert need > 0
    ws = torch.empty(need // 4 + 1, dtype=torch.float32, device=DEV)
    ref = run(xi, vi, xj, vj, mj, 0.1)
    got = run(xi, vi, xj, vj, mj, 0.1, workspace=ws)
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)
