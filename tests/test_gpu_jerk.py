"""GPU parity of the force-jerk-potential path (nbody_force_jerk*) against the oracle.

Both sides see the same seeded particles (FP32 values promoted to FP64 for the
oracle).  Acceleration and potential use the force path's bounds (relative RMS
<= 1e-6 compensated / FP64-reduced).  The jerk sums terms of both signs whose sizes
are set by relative velocities, so its per-particle relative error scales with the
condition number sum|term| / |sum term|.  The test therefore bounds each particle's
error by the arithmetic.  With B_ij = m_j (|w| / s^3 + 3 |d.w| |d| / s^5), a
worst-case count of the FP32 roundings in one pair term (separations u, s^2 2u,
rsq about 2u, m/s^3 about 9u, d.w 4u |d||w|, the bracket w - 3 (d.w / s^2) d up to
38u |w|) gives |Delta term| <= 74 u B_ij, so |Delta jerk_i| <= 74 u sum_j B_ij
(u = 2^-24).  The sums add at most (A - 1) u sum_j B_ij more, A the longest run of
FP32 additions: one compensation block (128 j's) in the compensated and FP64-reduced
modes, the segment plus the segment sum (< n + 1024) in plain FP32.  Relative RMS and
normwise errors are reported beside the bound.
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
U = 2.0 ** -24
TOL = {"comp": 1e-6, "fp64red": 1e-6, "plain": 1e-5}
C_JERK = 74.0
BLOCK_J = 128  # FP32 additions per compensation block


def as32(a):
    return a.astype(np.float32).astype(np.float64)


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a.T.astype(dtype))).to(DEV)


def run(x, v, m, eps, **kw):
    acc, jerk, pot = api.force_jerk(dev(x), dev(v), torch.from_numpy(m.astype(np.float32)).to(DEV),
                                    eps, **kw)
    torch.cuda.synchronize()
    return acc.cpu().numpy().T, jerk.cpu().numpy().T, pot.cpu().numpy() if pot is not None else None


def jerk_scale(x, v, m, eps, idx):
    """sum_j B_ij for the listed i (FP64, numpy; j == i contributes 0)."""
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        d = x - x[i]
        w = v - v[i]
        s2 = (d * d).sum(1) + eps * eps
        s = np.sqrt(s2)
        dw = np.abs((d * w).sum(1))
        b = m * (np.sqrt((w * w).sum(1)) / (s2 * s) + 3 * dw * np.sqrt((d * d).sum(1)) / (s2 * s2 * s))
        out[t] = b.sum()
    return out


def check_jerk_bound(jerk, ref, scale, precision, n):
    err = np.sqrt(((jerk - ref) ** 2).sum(1))
    c = C_JERK + (n + 1024 if precision == "plain" else BLOCK_J - 1)
    ratio = err / (U * scale)
    assert np.all(ratio <= c), (precision, float(ratio.max()))
    return float(ratio.max())


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_plummer_2048_full_parity(precision):
    n = 2048
    x, v, m = ics.plummer(n, seed=1)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(1.0 / 64))
    acc, jerk, pot = run(x, v, m, eps, precision=precision)
    ra, rj, rp = oracle.force_jerk(x, v, m, eps)
    ea, ej, ep = rel_errors(acc, ra), rel_errors(jerk, rj), rel_errors(pot, rp)
    idx = np.arange(n)
    worst = check_jerk_bound(jerk, rj, jerk_scale(x, v, m, eps, idx), precision, n)
    print(precision, "acc", ea, "jerk", ej, "pot", ep, "jerk err / (u sum B) max %.2f" % worst)
    assert ea["rel_rms"] <= TOL[precision], ea
    assert ep["rel_rms"] <= TOL[precision], ep
    assert ej["normwise"] <= 10 * TOL[precision], ej


@pytest.mark.parametrize("n", [1, 2, 3, 63, 255, 257, 1025, 3001])
def test_ragged_sizes(n):
    x, v, m = ics.plummer(n, seed=400 + n)
    m = m * np.random.default_rng(n).uniform(0.5, 1.5, n)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(0.03))
    ra, rj, rp = oracle.force_jerk(x, v, m, eps)
    for precision in ("comp", "plain"):
        acc, jerk, pot = run(x, v, m, eps, precision=precision)
        if n == 1:
            assert np.all(acc == 0) and np.all(jerk == 0) and np.all(pot == 0)
            continue
        assert rel_errors(acc, ra)["rel_rms"] <= TOL[precision]
        check_jerk_bound(jerk, rj, jerk_scale(x, v, m, eps, np.arange(n)), precision, n)
        # Potential terms share a sign, so sum |term| = |phi|: each term's rounding (the
        # product m rsq(s^2), C_POT u) and the FP32 additions after it (a 128-term block;
        # plain: the segment and the segment sum) bound every particle's error.
        worst = bounds.check_pot(pot, rp, np.abs(rp), precision, n)
        print(precision, n, "pot err / (u |phi|) max %.2f" % worst)


@pytest.mark.parametrize("ipl,jtile,nseg", [(1, 64, 1), (2, 128, 7), (4, 256, 3), (8, 512, 2),
                                             (1, 512, 40)])
def test_launch_shapes(ipl, jtile, nseg):
    n = 4000
    x, v, m = ics.plummer(n, seed=17)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(0.02))
    ra, rj, _ = oracle.force_jerk(x, v, m, eps)
    acc, jerk, _ = run(x, v, m, eps, precision="comp", ipl=ipl, jtile=jtile, nseg=nseg)
    assert rel_errors(acc, ra)["rel_rms"] <= 1e-6
    assert rel_errors(jerk, rj)["normwise"] <= 1e-5


def test_two_body_and_self_potential():
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    v = np.array([[0.0, 0.0, 0.0], [0.5, -1.0, 0.25]])
    m = np.array([0.25, 0.5])
    acc, jerk, pot = run(x, v, m, 4.0, precision="comp")
    ra, rj, rp = oracle.force_jerk(x, v, m, 4.0)
    np.testing.assert_allclose(acc, ra, rtol=1e-6)
    np.testing.assert_allclose(jerk, rj, rtol=2e-6)
    np.testing.assert_allclose(pot, rp, rtol=1e-6)
    a_self, j_self, pot_self = run(x, v, m, 4.0, precision="comp", self_pot=True)
    # The self term -m_i/eps is added in FP64 to the same sums.
    np.testing.assert_array_equal(a_self, acc)
    np.testing.assert_array_equal(j_self, jerk)
    np.testing.assert_array_equal(pot_self, pot - m / 4.0)


def test_fp64_state_with_centres():
    # A cluster far from the origin moving fast: the FP64 entry point takes positions and
    # velocities relative to their FP64 means (per system, or per i-tile after a Morton
    # sort); the plain FP32 rounding loses digits.
    n = 3000
    x, v, m = ics.plummer(n, seed=23)
    x = x + np.array([200.0, -50.0, 10.0])
    v = v + np.array([40.0, 0.0, -20.0])
    perm = api.morton_order(dev(x, np.float64)).cpu().numpy().astype(np.int64)
    x, v, m = x[perm], v[perm], m[perm]
    m32 = m.astype(np.float32)
    eps = float(np.float32(0.02))
    ra, rj, rp = oracle.force_jerk(x, v, m32.astype(np.float64), eps)
    mt = torch.from_numpy(m32).to(DEV)
    errs = {}
    for centre in ("tile", "system", "none"):
        acc, jerk, pot = api.force_jerk(dev(x, np.float64), dev(v, np.float64), mt, eps,
                                        centre=centre)
        torch.cuda.synchronize()
        errs[centre] = (rel_errors(acc.cpu().numpy().T, ra), rel_errors(jerk.cpu().numpy().T, rj),
                        rel_errors(pot.cpu().numpy(), rp))
        print(centre, errs[centre])
    for centre in ("tile", "system"):
        assert errs[centre][0]["rel_rms"] <= 1e-6
        assert errs[centre][1]["normwise"] <= 1e-5
        assert errs[centre][2]["rel_rms"] <= 1e-6
    # (Tile centres only beat the system centre when tiles are much smaller than the
    # system, as in a dense core; for one sphere both conversions err by about u |x|.)
    assert errs["none"][1]["normwise"] > 10 * errs["system"][1]["normwise"]


def test_paper_scale_sampled():
    # N = 131072 Plummer with distribution-function velocities (the paper quotes its
    # force-jerk rate at this N); 1024 sampled i's against the oracle.
    w = ics.WORKLOADS["plummer_131072"]
    x, v, m = ics.plummer(w.n, seed=w.seed)
    x, v, m = as32(x), as32(v), as32(m)
    eps = float(np.float32(w.eps))
    acc, jerk, pot = run(x, v, m, eps, precision="comp")
    idx = ics.sample_indices(w.n, 1024, seed=w.seed + 1000)
    ra, rj, rp = oracle.force_jerk(x, v, m, eps, idx=idx)
    ea, ej, ep = rel_errors(acc[idx], ra), rel_errors(jerk[idx], rj), rel_errors(pot[idx], rp)
    worst = check_jerk_bound(jerk[idx], rj, jerk_scale(x, v, m, eps, idx), "comp", w.n)
    print("acc", ea, "jerk", ej, "pot", ep, "bound ratio", worst)
    assert ea["rel_rms"] <= 1e-6, ea
    assert ep["rel_rms"] <= 1e-6, ep
    assert ej["normwise"] <= 1e-5, ej


def test_caller_workspace_gives_identical_results():
    n = 1500
    x, v, m = ics.plummer(n, seed=29)
    need = _lib.nbody_workspace_size_jerk(n, None)
    assert need > 0
    ws = torch.empty(need // 4, dtype=torch.float32, device=DEV)
    a1, j1, _ = run(x, v, m, 0.05, precision="comp", workspace=ws)
    a2, j2, _ = run(x, v, m, 0.05, precision="comp")
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(j1, j2)
