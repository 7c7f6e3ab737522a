"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the property it relies on.  A plausible slip in the oracle (a
dropped term, a wrong sign or power, a transposed index, a missing self
exclusion) fails at least one of them.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
from paper_astro_ph_0703100_amd import ics
from paper_astro_ph_0703100_amd.metrics import rel_errors
from conftest import load_golden


# --------------------------------------------------------------------------- closed forms
def test_two_body_closed_form():
    # d = (1, 2, 2) has |d| = 3; with eps = 4 the softened distance is exactly 5, so
    # a_1 = m_2 d / 125 and phi_1 = -m_2 / 5 (eq. (1)); a_2, phi_2 mirror it with m_1.
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    m = np.array([0.25, 0.5])
    acc, pot = oracle.force_all(x, m, 4.0)
    np.testing.assert_allclose(acc[0], [0.004, 0.008, 0.008], rtol=2e-16, atol=0)
    np.testing.assert_allclose(acc[1], [-0.002, -0.004, -0.004], rtol=2e-16, atol=0)
    np.testing.assert_allclose(pot, [-0.1, -0.05], rtol=2e-16, atol=0)


def test_two_body_axis_and_shift():
    # Separation 3 along z, eps = 4 -> distance 5; translating both bodies changes nothing
    # (up to rounding of the shifted coordinates, which are exact here).
    x = np.array([[10.0, -4.0, 7.0], [10.0, -4.0, 10.0]])
    m = np.array([2.0, 1.0])
    acc, pot = oracle.force_all(x, m, 4.0)
    np.testing.assert_allclose(acc, [[0, 0, 3.0 / 125.0], [0, 0, -6.0 / 125.0]], rtol=2e-16, atol=0)
    np.testing.assert_allclose(pot, [-0.2, -0.4], rtol=2e-16)


def test_coincident_pair_and_single_particle():
    # Two particles at the same place: no force, potential -m_other / eps.
    x = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    acc, pot = oracle.force_all(x, np.array([1.0, 3.0]), 0.25)
    assert np.all(acc == 0.0)
    np.testing.assert_array_equal(pot, [-12.0, -4.0])
    # One particle: nothing acts on it (self pair excluded).
    acc, pot = oracle.force_all(np.array([[1.0, 2.0, 3.0]]), np.array([1.0]), 0.1)
    assert np.all(acc == 0.0) and np.all(pot == 0.0)
    # Empty input.
    acc, pot = oracle.force_all(np.zeros((0, 3)), np.zeros(0), 0.1)
    assert acc.shape == (0, 3) and pot.shape == (0,)


def _decimal_force(x, m, eps, digits=50):
    """Brute-force sum in 50-digit decimal arithmetic (stdlib Decimal.sqrt)."""
    getcontext().prec = digits
    n = len(m)
    X = [[Decimal(float(v)) for v in row] for row in x]
    M = [Decimal(float(v)) for v in m]
    e2 = Decimal(float(eps)) ** 2
    acc = []
    pot = []
    for i in range(n):
        a = [Decimal(0)] * 3
        p = Decimal(0)
        for j in range(n):
            if j == i:
                continue
            d = [X[j][c] - X[i][c] for c in range(3)]
            s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2
            s = s2.sqrt()
            for c in range(3):
                a[c] += M[j] * d[c] / (s2 * s)
            p -= M[j] / s
        acc.append([float(v) for v in a])
        pot.append(float(p))
    return np.array(acc), np.array(pot)


@pytest.mark.parametrize("n,seed", [(2, 1), (5, 2), (9, 3), (16, 4)])
def test_tiny_n_against_decimal(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    m = rng.uniform(0.1, 1.0, n)
    acc, pot = oracle.force_all(x, m, 0.05)
    ea, ep = _decimal_force(x, m, 0.05)
    assert rel_errors(acc, ea)["e_max"] < 1e-13
    assert rel_errors(pot, ep)["e_max"] < 1e-14


# --------------------------------------------------------------------------- invariants
def test_momentum_conservation():
    # Pairwise antisymmetry of eq. (1): sum_i m_i a_i = 0.
    x, _, m = ics.plummer(1024, seed=7)
    m = m * np.random.default_rng(8).uniform(0.5, 1.5, m.size)
    acc, _ = oracle.force_all(x, m, 0.01)
    resid = np.abs((m[:, None] * acc).sum(0))
    scale = (m[:, None] * np.abs(acc)).sum(0)
    assert np.all(resid < 1e-14 * scale)


def test_power_of_two_scaling_is_exact():
    # x -> 2^k x and eps -> 2^k eps scale a by 2^-2k and phi by 2^-k with no rounding
    # change; m -> 2^k m scales both by 2^k.
    x, _, m = ics.plummer(256, seed=9)
    acc, pot = oracle.force_all(x, m, 0.02)
    acc2, pot2 = oracle.force_all(x * 8.0, m, 0.16)
    np.testing.assert_array_equal(acc2, acc / 64.0)
    np.testing.assert_array_equal(pot2, pot / 8.0)
    acc3, pot3 = oracle.force_all(x, m * 0.25, 0.02)
    np.testing.assert_array_equal(acc3, acc * 0.25)
    np.testing.assert_array_equal(pot3, pot * 0.25)


def test_permutation_equivariance():
    x, _, m = ics.plummer(300, seed=10)
    perm = np.random.default_rng(3).permutation(300)
    acc, pot = oracle.force_all(x, m, 0.01)
    accp, potp = oracle.force_all(x[perm], m[perm], 0.01)
    np.testing.assert_allclose(accp, acc[perm], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(potp, pot[perm], rtol=1e-13)


def test_sampled_and_ij_forms_agree_with_all_pairs():
    x, _, m = ics.plummer(700, seed=12)
    acc, pot = oracle.force_all(x, m, 0.03)
    idx = np.array([0, 5, 699, 350])
    a2, p2 = oracle.force_sampled(x, m, 0.03, idx)
    np.testing.assert_array_equal(a2, acc[idx])
    np.testing.assert_array_equal(p2, pot[idx])
    a3, p3 = oracle.force_ij(x, m, x[idx], 0.03, self_index=idx)
    np.testing.assert_array_equal(a3, acc[idx])
    # Separate i-set (no exclusion) adds the self term -m_i/eps to phi and nothing to a.
    a4, p4 = oracle.force_ij(x, m, x[idx], 0.03)
    np.testing.assert_allclose(a4, acc[idx], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(p4, pot[idx] - m[idx] / 0.03, rtol=1e-13)


def test_separate_sets_with_per_i_softening_closed_form():
    # j at (1, 2, 2) (|d| = 3) with mass 0.5, seen from three i-particles at the origin
    # with eps = 4, 0 and 0 (the last one shifted to (1, 2, 0): |d| = 2):
    # a = m d / (|d|^2 + eps^2)^{3/2}, phi = -m / sqrt(|d|^2 + eps^2).
    xj = np.array([[1.0, 2.0, 2.0]])
    mj = np.array([0.5])
    xi = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 2.0, 0.0]])
    acc, pot = oracle.force_ij(xj, mj, xi, None, eps_i=np.array([4.0, 0.0, 0.0]))
    np.testing.assert_allclose(acc[0], [0.5 / 125, 1.0 / 125, 1.0 / 125], rtol=2e-16, atol=0)
    np.testing.assert_allclose(acc[1], [0.5 / 27, 1.0 / 27, 1.0 / 27], rtol=2e-16, atol=0)
    np.testing.assert_allclose(acc[2], [0.0, 0.0, 1.0 / 8], rtol=2e-16, atol=0)
    np.testing.assert_allclose(pot, [-0.1, -0.5 / 3, -0.25], rtol=2e-16)
    # No j-particles: zeros.
    acc, pot = oracle.force_ij(np.zeros((0, 3)), np.zeros(0), xi, None, eps_i=np.ones(3))
    assert np.all(acc == 0.0) and np.all(pot == 0.0)


def test_separate_sets_with_per_i_softening_against_decimal():
    rng = np.random.default_rng(21)
    xi, xj = rng.standard_normal((7, 3)), rng.standard_normal((11, 3))
    mj = rng.uniform(0.1, 1.0, 11)
    eps_i = rng.uniform(0.0, 0.3, 7)
    eps_i[2] = 0.0
    acc, pot = oracle.force_ij(xj, mj, xi, None, eps_i=eps_i)
    getcontext().prec = 50
    for i in range(7):
        a = [Decimal(0)] * 3
        p = Decimal(0)
        e2 = Decimal(float(eps_i[i])) ** 2
        for j in range(11):
            d = [Decimal(float(xj[j, c])) - Decimal(float(xi[i, c])) for c in range(3)]
            s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2
            s = s2.sqrt()
            for c in range(3):
                a[c] += Decimal(float(mj[j])) * d[c] / (s2 * s)
            p -= Decimal(float(mj[j])) / s
        np.testing.assert_allclose(acc[i], [float(v) for v in a], rtol=1e-13)
        assert abs(pot[i] - float(p)) <= 1e-14 * abs(float(p))


# --------------------------------------------------------------------------- jerk
def test_jerk_two_body_closed_form():
    # d = (1, 2, 2), eps = 4: s = 5; w = v_2 - v_1 = (0.5, -1, 0.25), d.w = -1, so
    # jerk_1 = m_2 (w / 125 + 3 d / 3125) and jerk_2 = -m_1 (w / 125 + 3 d / 3125).
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    v = np.array([[0.0, 0.0, 0.0], [0.5, -1.0, 0.25]])
    m = np.array([0.25, 0.5])
    acc, jerk, pot = oracle.force_jerk(x, v, m, 4.0)
    base = np.array([0.004 + 0.00096, -0.008 + 0.00192, 0.002 + 0.00192])
    np.testing.assert_allclose(jerk[0], 0.5 * base, rtol=1e-15, atol=0)
    np.testing.assert_allclose(jerk[1], -0.25 * base, rtol=1e-15, atol=0)
    np.testing.assert_allclose(acc[0], [0.004, 0.008, 0.008], rtol=2e-16, atol=0)
    np.testing.assert_allclose(pot, [-0.1, -0.05], rtol=2e-16)


def test_jerk_is_the_time_derivative_of_the_force():
    # Along straight-line motion x(t) = x + v t, jerk = d a / dt; central differences
    # of the (separately pinned) force sum, h = 1e-5, truncation error O(h^2).
    x, v, m = ics.plummer(64, seed=31)
    eps, h = 0.05, 1e-5
    _, jerk, _ = oracle.force_jerk(x, v, m, eps)
    ap, _ = oracle.force_all(x + h * v, m, eps)
    am, _ = oracle.force_all(x - h * v, m, eps)
    fd = (ap - am) / (2 * h)
    assert rel_errors(jerk, fd)["normwise"] < 1e-8
    assert rel_errors(jerk, fd)["rel_rms"] < 1e-7


def test_jerk_against_decimal():
    rng = np.random.default_rng(33)
    n = 6
    x, v = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    m = rng.uniform(0.1, 1.0, n)
    eps = 0.1
    _, jerk, _ = oracle.force_jerk(x, v, m, eps)
    getcontext().prec = 50
    D = lambda a: Decimal(float(a))
    for i in range(n):
        jk = [Decimal(0)] * 3
        for j in range(n):
            if j == i:
                continue
            d = [D(x[j, c]) - D(x[i, c]) for c in range(3)]
            w = [D(v[j, c]) - D(v[i, c]) for c in range(3)]
            s2 = sum(t * t for t in d) + D(eps) ** 2
            s = s2.sqrt()
            dw = sum(d[c] * w[c] for c in range(3))
            for c in range(3):
                jk[c] += D(m[j]) * (w[c] / (s2 * s) - 3 * dw * d[c] / (s2 * s2 * s))
        np.testing.assert_allclose(jerk[i], [float(t) for t in jk], rtol=1e-12, atol=1e-14)


def test_jerk_invariants():
    x, v, m = ics.plummer(500, seed=35)
    m = m * np.random.default_rng(36).uniform(0.5, 1.5, m.size)
    acc, jerk, pot = oracle.force_jerk(x, v, m, 0.02)
    # sum_i m_i jerk_i = d/dt sum_i m_i a_i = 0 (pairwise antisymmetry).
    resid = np.abs((m[:, None] * jerk).sum(0))
    assert np.all(resid < 1e-13 * (m[:, None] * np.abs(jerk)).sum(0))
    # v -> 4 v scales the jerk exactly and leaves a and phi alone.
    a4, j4, p4 = oracle.force_jerk(x, 4.0 * v, m, 0.02)
    np.testing.assert_array_equal(j4, 4.0 * jerk)
    np.testing.assert_array_equal(a4, acc)
    np.testing.assert_array_equal(p4, pot)
    # A common velocity changes nothing but rounding (Galilean invariance).
    _, jg, _ = oracle.force_jerk(x, v + np.array([0.3, -0.2, 0.1]), m, 0.02)
    assert rel_errors(jg, jerk)["normwise"] < 1e-13
    # The force and potential agree with the force-only sum; a sample agrees with the whole.
    af, pf = oracle.force_all(x, m, 0.02)
    np.testing.assert_array_equal(acc, af)
    np.testing.assert_array_equal(pot, pf)
    idx = np.array([3, 0, 499])
    a_s, j_s, p_s = oracle.force_jerk(x, v, m, 0.02, idx=idx)
    np.testing.assert_array_equal(j_s, jerk[idx])


def test_jerk_ij_is_the_time_derivative_of_force_ij():
    # Separate sets in relative motion (an active subset of one sphere against another
    # sphere): along x_i + v_i t and x_j + v_j t the jerk is d a_i / dt; central
    # differences of the (separately pinned) force_ij, h = 1e-5, with eps = 0 as well.
    xj, vj, mj = ics.plummer(80, seed=37)
    xi, vi, _ = ics.plummer(20, seed=38)
    xi = xi * 0.7 + 0.3
    h = 1e-5
    for eps in (0.05, 0.0):
        _, jerk, _ = oracle.force_jerk_ij(xj, vj, mj, xi, vi, eps)
        ap, _ = oracle.force_ij(xj + h * vj, mj, xi + h * vi, eps)
        am, _ = oracle.force_ij(xj - h * vj, mj, xi - h * vi, eps)
        fd = (ap - am) / (2 * h)
        assert rel_errors(jerk, fd)["normwise"] < 1e-7, eps


def test_jerk_ij_on_one_set_matches_force_jerk():
    # With the i-set equal to the j-set the only difference from the single-set sum is
    # the j == i pair: it adds exactly zero to a and the jerk and -m_i/eps to phi.
    x, v, m = ics.plummer(300, seed=39)
    m = m * np.random.default_rng(40).uniform(0.5, 1.5, m.size)
    eps = 0.03
    a1, j1, p1 = oracle.force_jerk(x, v, m, eps)
    a2, j2, p2 = oracle.force_jerk_ij(x, v, m, x, v, eps)
    np.testing.assert_array_equal(a2, a1)
    np.testing.assert_array_equal(j2, j1)
    np.testing.assert_allclose(p2, p1 - m / eps, rtol=1e-13)


# --------------------------------------------------------------------------- mean field
def test_shell_theorem_on_plummer_realisation():
    # For a near-spherical particle set the shell-averaged field at radius r is that of
    # the realised shells: a_r = -M(<r)/r^2 and phi = -M(<r)/r - sum_{r_j>r} m_j/r_j.
    # Bin means of the per-particle ratios must be 1 within the anisotropy noise.
    n = 16384
    pos, _, mass = ics.plummer(n, seed=11, velocities=False)
    idx = ics.sample_indices(n, 2048, seed=12)
    acc, pot = oracle.force_sampled(pos, mass, 1e-3, idx)
    rall = np.linalg.norm(pos, axis=1)
    order = np.argsort(rall)
    rs, ms = rall[order], mass[order]
    cm = np.cumsum(ms)
    tail = np.cumsum((ms / rs)[::-1])[::-1]
    r = rall[idx]
    k = np.searchsorted(rs, r)
    menc = cm[k] - mass[idx]
    outside = np.where(k + 1 < n, tail[np.minimum(k + 1, n - 1)], 0.0)
    ratio_a = ((acc * pos[idx]).sum(1) / r) / (-menc / r ** 2)
    ratio_p = pot / (-menc / r - outside)
    for lo, hi in [(0.3, 0.6), (0.6, 1.0), (1.0, 2.0), (2.0, 4.0), (4.0, 10.0)]:
        s = (r >= lo) & (r < hi)
        sa = ratio_a[s].std() / math.sqrt(s.sum())
        assert abs(ratio_a[s].mean() - 1.0) < 4 * sa + 2e-3, (lo, hi, ratio_a[s].mean(), sa)
        assert abs(ratio_p[s].mean() - 1.0) < 2e-3, (lo, hi, ratio_p[s].mean())


def test_plummer_analytic_mean_field():
    # Truncated Plummer model (scale 1, truncation R = 20, total mass 1):
    # a(r) = -M(r)/(M(R) r^2), phi(r) = [-(1+r^2)^-1/2 + (1+R^2)^-1/2 - M(R)/R] / M(R),
    # M(r) = r^3/(1+r^2)^{3/2}.  Discreteness noise at N = 16384 is a few per cent.
    n = 16384
    pos, _, mass = ics.plummer(n, seed=21, velocities=False)
    idx = ics.sample_indices(n, 2048, seed=22)
    acc, pot = oracle.force_sampled(pos, mass, 1e-3, idx)
    R = 20.0
    MR = R ** 3 / (1 + R * R) ** 1.5
    r = np.linalg.norm(pos[idx], axis=1)
    ar = (acc * pos[idx]).sum(1) / r
    a_model = -(r ** 3 / (1 + r * r) ** 1.5) / MR / r ** 2
    p_model = (-(1 + r * r) ** -0.5 + (1 + R * R) ** -0.5 - MR / R) / MR
    s = (r > 0.3) & (r < 10)
    assert abs(np.mean(ar[s] / a_model[s]) - 1) < 0.03
    assert abs(np.mean(pot[s] / p_model[s]) - 1) < 0.01


# --------------------------------------------------------------------------- Table 2
@pytest.mark.parametrize("n", [2048, 4096, 8192])
def test_table2_error_magnitudes(n):
    # Replaying the paper's two FP32 accumulation orders against the FP64 oracle on the
    # same FP32-rounded particles gives E_max of the magnitude printed in Table 2
    # (standard N-body units, eps^2 = 0.01, J-BAG of 512).  Our spheres are other
    # realisations, so only the magnitude is compared: DIRECT within 2x, the J-BAG
    # order within 4x, and the J-BAG order better than DIRECT.
    table = load_golden("table2_cumulative_error.txt")
    row = table[table[:, 0] == n][0]
    pos, _, m = ics.nemo_plummer(n, seed=100 + n)
    x32 = pos.astype(np.float32)
    m32 = m.astype(np.float32)
    idx = np.arange(n)
    ref, _ = oracle.force_sampled(x32.astype(np.float64), m32.astype(np.float64), 0.1, idx)
    direct = rel_errors(oracle.fp32_replay(x32, m32, np.float32(0.01), 0, idx), ref)["e_max"]
    bag = rel_errors(oracle.fp32_replay(x32, m32, np.float32(0.01), 512, idx), ref)["e_max"]
    assert row[1] / 2 < direct < row[1] * 2, (direct, row[1])
    assert row[2] / 4 < bag < row[2] * 4, (bag, row[2])
    assert bag < direct


# --------------------------------------------------------------------------- VJP
def _scalar_loss(x, m, eps, ga, gp):
    acc, pot = oracle.force_all(x, m, eps)
    return float((acc * ga).sum() + (pot * gp).sum())


def test_vjp_against_central_differences():
    rng = np.random.default_rng(31)
    n = 20
    x = rng.standard_normal((n, 3))
    m = rng.uniform(0.2, 1.0, n)
    eps = 0.3
    ga = rng.standard_normal((n, 3))
    gp = rng.standard_normal(n)
    gx, gm = oracle.vjp(x, m, eps, ga, gp)
    h = 1e-6
    fd_x = np.empty_like(x)
    for k in range(n):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fd_x[k, c] = (_scalar_loss(xp, m, eps, ga, gp) - _scalar_loss(xm, m, eps, ga, gp)) / (2 * h)
    fd_m = np.empty(n)
    for k in range(n):
        mp, mm = m.copy(), m.copy()
        mp[k] += h
        mm[k] -= h
        fd_m[k] = (_scalar_loss(x, mp, eps, ga, gp) - _scalar_loss(x, mm, eps, ga, gp)) / (2 * h)
    assert np.linalg.norm(gx - fd_x) / np.linalg.norm(fd_x) < 1e-8
    assert np.linalg.norm(gm - fd_m) / np.linalg.norm(fd_m) < 1e-8
    # Without a potential cotangent.
    gx0, gm0 = oracle.vjp(x, m, eps, ga, None)
    gx1, gm1 = oracle.vjp(x, m, eps, ga, np.zeros(n))
    np.testing.assert_array_equal(gx0, gx1)
    np.testing.assert_array_equal(gm0, gm1)


def test_vjp_invariants():
    # Translation invariance of a and phi: sum_k dL/dx_k = 0.
    # Degree-1 homogeneity in m: sum_k m_k dL/dm_k = sum_i ga_i.a_i + gp_i phi_i.
    x, _, m = ics.plummer(512, seed=33)
    rng = np.random.default_rng(34)
    m = m * rng.uniform(0.5, 1.5, m.size)
    ga = rng.standard_normal(x.shape)
    gp = rng.standard_normal(m.size)
    gx, gm = oracle.vjp(x, m, 0.02, ga, gp)
    assert np.all(np.abs(gx.sum(0)) < 1e-12 * np.abs(gx).sum(0))
    acc, pot = oracle.force_all(x, m, 0.02)
    lhs = float((m * gm).sum())
    rhs = float((ga * acc).sum() + (gp * pot).sum())
    assert abs(lhs - rhs) < 1e-12 * (abs(rhs) + np.abs(m * gm).sum())


# --------------------------------------------------------------------------- integrator
def test_two_body_circular_orbit():
    # Equal masses 1/2 at separation 1: each moves on a circle of radius 1/2 with
    # omega^2 = (1 + eps^2)^{-3/2}; after one period both are back where they started
    # (to the leapfrog's O(dt^2) phase error).
    eps = 0.01
    om = (1 + eps * eps) ** -0.75
    x0 = np.array([[0.5, 0, 0], [-0.5, 0, 0]])
    v0 = np.array([[0, 0.5 * om, 0], [0, -0.5 * om, 0]])
    m = np.array([0.5, 0.5])
    period = 2 * math.pi / om
    for nsteps, tol in ((2000, 2e-5), (4000, 5e-6)):
        x, v, _, _ = oracle.rollout(x0, v0, m, eps, period / nsteps, nsteps)
        err = np.abs(x - x0).max()
        assert err < tol, (nsteps, err)
    # Radius stays 1/2 along the way.
    _, _, _, traj = oracle.rollout(x0, v0, m, eps, period / 400, 100, keep_trajectory=True)
    sep = np.linalg.norm(traj[:, 0] - traj[:, 1], axis=1)
    assert np.abs(sep - 1.0).max() < 1e-4


def test_hermite_circular_orbit_fourth_order():
    # The two-body circular orbit above, integrated with the fourth-order Hermite scheme:
    # the position error after one period falls by about 2^4 when dt halves, and is far
    # below the leapfrog's at the same step.
    eps = 0.01
    om = (1 + eps * eps) ** -0.75
    x0 = np.array([[0.5, 0, 0], [-0.5, 0, 0]])
    v0 = np.array([[0, 0.5 * om, 0], [0, -0.5 * om, 0]])
    m = np.array([0.5, 0.5])
    period = 2 * math.pi / om
    errs = []
    for nsteps in (100, 200):
        x, v, _, _ = oracle.hermite(x0, v0, m, eps, period / nsteps, nsteps)
        errs.append(np.abs(x - x0).max())
    assert 11 < errs[0] / errs[1] < 22, errs
    xl, _, _, _ = oracle.rollout(x0, v0, m, eps, period / 200, 200)
    assert errs[1] < 0.01 * np.abs(xl - x0).max()
    # One step against the exact rotation by omega dt: a fourth-order scheme has local
    # errors O(dt^5) in both position and velocity (ratio about 32 when dt halves).
    loc = []
    for dt in (0.1, 0.05):
        x, v, _, _ = oracle.hermite(x0, v0, m, eps, dt, 1)
        c, s_ = math.cos(om * dt), math.sin(om * dt)
        xe = np.array([[0.5 * c, 0.5 * s_, 0], [-0.5 * c, -0.5 * s_, 0]])
        ve = np.array([[-0.5 * om * s_, 0.5 * om * c, 0], [0.5 * om * s_, -0.5 * om * c, 0]])
        loc.append((np.abs(x - xe).max(), np.abs(v - ve).max()))
    assert 24 < loc[0][0] / loc[1][0] < 40, loc
    assert 24 < loc[0][1] / loc[1][1] < 40, loc


def test_hermite_energy_order_and_leapfrog_limit():
    x0, v0, m = ics.plummer(48, seed=43)
    eps, T = 0.05, 0.25

    def energy_err(nsteps):
        x, v, _, _ = oracle.hermite(x0, v0, m, eps, T / nsteps, nsteps)
        return abs(oracle.energy(x, v, m, eps) - oracle.energy(x0, v0, m, eps))

    e1, e2 = energy_err(32), energy_err(64)
    assert 8 < e1 / e2 < 40, (e1, e2)
    # Both integrators converge to the same trajectory.
    xh, vh, _, _ = oracle.hermite(x0, v0, m, eps, T / 256, 256)
    xl, vl, _, _ = oracle.rollout(x0, v0, m, eps, T / 4096, 4096)
    assert np.abs(xh - xl).max() < 1e-7
    assert np.abs(vh - vl).max() < 1e-6
    # Free motion is exact: one particle moves in a straight line.
    x, v, a, j = oracle.hermite(np.array([[1.0, 2.0, 3.0]]), np.array([[0.5, -0.25, 2.0]]),
                                np.array([1.0]), 0.1, 0.125, 8)
    np.testing.assert_array_equal(x, [[1.5, 1.75, 5.0]])
    assert np.all(a == 0) and np.all(j == 0)


def test_leapfrog_time_reversibility_and_energy_order():
    x0, v0, m = ics.plummer(64, seed=41)
    eps = 0.05
    x, v, _, _ = oracle.rollout(x0, v0, m, eps, 1.0 / 128, 64)
    xb, vb, _, _ = oracle.rollout(x, -v, m, eps, 1.0 / 128, 64)
    assert np.abs(xb - x0).max() < 1e-11
    assert np.abs(vb + v0).max() < 1e-11
    e0 = oracle.energy(x0, v0, m, eps)
    errs = []
    for dt in (1.0 / 32, 1.0 / 64):
        xx, vv, _, _ = oracle.rollout(x0, v0, m, eps, dt, int(round(0.5 / dt)))
        errs.append(abs(oracle.energy(xx, vv, m, eps) - e0))
    ratio = errs[0] / errs[1]
    assert 2.5 < ratio < 6.0, ratio


def test_rollout_gradient_against_central_differences():
    n, steps, dt, eps = 12, 6, 1.0 / 64, 0.1
    x0, v0, m = ics.plummer(n, seed=51)
    m = m * np.random.default_rng(52).uniform(0.5, 1.5, n)
    y = ics.perturbed_target(x0, seed=53, scale=0.05)
    loss, gx, gv, gm = oracle.rollout_loss_grad(x0, v0, m, eps, dt, steps, y)

    def L(x, v, mm):
        xT, _, _, _ = oracle.rollout(x, v, mm, eps, dt, steps)
        return float(np.sum((xT - y) ** 2) / n)

    assert abs(L(x0, v0, m) - loss) < 1e-15 * max(1.0, loss)
    h = 1e-6
    rng = np.random.default_rng(54)
    for _ in range(8):
        k, c = int(rng.integers(n)), int(rng.integers(3))
        xp, xm = x0.copy(), x0.copy()
        xp[k, c] += h
        xm[k, c] -= h
        fd = (L(xp, v0, m) - L(xm, v0, m)) / (2 * h)
        assert abs(fd - gx[k, c]) < 1e-6 * np.abs(gx).max(), (k, c, fd, gx[k, c])
        vp, vm = v0.copy(), v0.copy()
        vp[k, c] += h
        vm[k, c] -= h
        fd = (L(x0, vp, m) - L(x0, vm, m)) / (2 * h)
        assert abs(fd - gv[k, c]) < 1e-6 * np.abs(gv).max()
    for k in range(0, n, 3):
        hm = 1e-6 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += hm
        mm[k] -= hm
        fd = (L(x0, v0, mp) - L(x0, v0, mm)) / (2 * hm)
        assert abs(fd - gm[k]) < 1e-6 * np.abs(gm).max(), (k, fd, gm[k])


@pytest.mark.parametrize("steps", [0, 1, 5])
def test_rollout_vjp_with_velocity_cotangent_against_central_differences(steps):
    # L = sum G . x_T + sum H . v_T: both final positions and final velocities carry a
    # cotangent.  Zero steps is the identity map (gradients G, H, 0); one step exercises
    # the two kicks of a single step.
    n, dt, eps = 10, 1.0 / 32, 0.1
    x0, v0, m = ics.plummer(n, seed=61)
    m = m * np.random.default_rng(62).uniform(0.5, 1.5, n)
    rng = np.random.default_rng(63)
    G, H = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    gx, gv, gm = oracle.rollout_vjp(x0, v0, m, eps, dt, steps, G, H)

    def L(x, v, mm):
        xT, vT, _, _ = oracle.rollout(x, v, mm, eps, dt, steps)
        return float(np.sum(G * xT) + np.sum(H * vT))

    if steps == 0:
        assert np.array_equal(gx, G) and np.array_equal(gv, H) and not gm.any()
    # A difference quotient carries the loss's rounding, a few u times the sum of the
    # magnitudes of its terms, divided by the step.
    xT, vT, _, _ = oracle.rollout(x0, v0, m, eps, dt, steps)
    mag = float(np.sum(np.abs(G * xT)) + np.sum(np.abs(H * vT)))
    noise = lambda step: 16 * 2.0 ** -53 * mag / step
    h = 1e-6
    for k in range(n):
        for c in range(3):
            xp, xm = x0.copy(), x0.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fd = (L(xp, v0, m) - L(xm, v0, m)) / (2 * h)
            assert abs(fd - gx[k, c]) < 1e-7 * np.abs(gx).max() + noise(h), (k, c, fd, gx[k, c])
            vp, vm = v0.copy(), v0.copy()
            vp[k, c] += h
            vm[k, c] -= h
            fd = (L(x0, vp, m) - L(x0, vm, m)) / (2 * h)
            assert abs(fd - gv[k, c]) < 1e-7 * np.abs(gv).max() + noise(h), (k, c, fd, gv[k, c])
        hm = 1e-6 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += hm
        mm[k] -= hm
        fd = (L(x0, v0, mp) - L(x0, v0, mm)) / (2 * hm)
        assert abs(fd - gm[k]) < 1e-7 * np.abs(gm).max() + noise(hm), (k, fd, gm[k])


def test_rollout_vjp_matches_the_loss_gradient():
    n, steps, dt, eps = 16, 4, 1.0 / 64, 0.1
    x0, v0, m = ics.plummer(n, seed=64)
    y = ics.perturbed_target(x0, seed=65, scale=0.05)
    loss, gx, gv, gm = oracle.rollout_loss_grad(x0, v0, m, eps, dt, steps, y)
    xT, _, _, _ = oracle.rollout(x0, v0, m, eps, dt, steps)
    rx, rv, rm = oracle.rollout_vjp(x0, v0, m, eps, dt, steps, 2.0 * (xT - y) / n, None)
    assert np.array_equal(rx, gx) and np.array_equal(rv, gv) and np.array_equal(rm, gm)


def test_force_abs_sums_pin():
    # j-particles all above-right-front of every i-particle (each separation component
    # positive) with positive masses: no term cancels, so the magnitude sums equal the
    # pinned force and potential; on a Plummer sphere they bound them, over the same
    # pairs as force_sampled.
    rng = np.random.default_rng(71)
    xi = rng.uniform(-1.0, 0.0, (20, 3))
    xj = rng.uniform(0.5, 2.0, (50, 3))
    mj = rng.uniform(0.1, 1.0, 50)
    absa, absp = oracle.force_abs(xj, mj, xi, 0.05)
    a, p = oracle.force_ij(xj, mj, xi, 0.05)
    np.testing.assert_allclose(absa, np.abs(a), rtol=1e-14)
    np.testing.assert_allclose(absp, np.abs(p), rtol=1e-14)
    x, _, m = ics.plummer(300, seed=72, velocities=False)
    idx = np.arange(0, 300, 7)
    absa, absp = oracle.force_abs_sampled(x, m, 0.02, idx)
    a, p = oracle.force_sampled(x, m, 0.02, idx)
    assert np.all(absa >= np.abs(a) * (1 - 1e-14)) and np.all(absa > 0)
    np.testing.assert_allclose(absp, np.abs(p), rtol=1e-13)
