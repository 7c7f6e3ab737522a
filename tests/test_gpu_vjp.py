"""GPU adjoint (VJP) and differentiable rollout against the FP64 oracle.

Tolerances: the adjoint sums terms of both signs (w = m_k g_j - m_j g_k) and the
cotangents are rounded to FP32 in the kernel, so its error is larger than the
force's.  dL/dx: relative RMS per particle <= 1e-5 and normwise <= 1e-6 for the
compensated and FP64-reduced modes.  dL/dm of a particle is a sum of terms of
random sign that can nearly cancel, so its per-particle relative error is
unbounded; it is held to normwise <= 1e-6 and to max |error| <= 1e-5 times the RMS
of dL/dm over all particles.  The rollout gradient: normwise <= 1e-4.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import _lib, api, autograd, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def setup(n, seed, eps=0.01, masses="equal"):
    pos, vel, mass = ics.plummer(n, seed=seed)
    if masses == "random":
        mass = mass * np.random.default_rng(seed).uniform(0.5, 1.5, n)
    m32 = mass.astype(np.float32)
    p32 = pos.astype(np.float32)
    rng = np.random.default_rng(seed + 1)
    ga = rng.standard_normal((n, 3))
    gp = rng.standard_normal(n)
    return p32, m32, ga, gp, vel


def scaled_max(approx, exact):
    """max_k |approx_k - exact_k| / RMS(exact)."""
    return float(np.abs(approx - exact).max() / np.sqrt(np.mean(exact ** 2)))


def gpu_vjp(p32, m32, eps, ga, gp, precision="comp", with_mass=True, **kw):
    n = len(m32)
    p = torch.from_numpy(np.ascontiguousarray(p32.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    g = torch.from_numpy(np.ascontiguousarray(ga.T)).to(DEV)
    gpt = torch.from_numpy(gp).to(DEV) if gp is not None else None
    gx = torch.empty((3, n), dtype=torch.float64, device=DEV)
    gm = torch.empty(n, dtype=torch.float64, device=DEV) if with_mass else None
    opts = api.make_opts(precision=precision, **kw)
    _lib.nbody_force_vjp(n, p.data_ptr(), m.data_ptr(), float(eps), g.data_ptr(),
                         gpt.data_ptr() if gpt is not None else None, gx.data_ptr(),
                         gm.data_ptr() if gm is not None else None, opts, api.stream_ptr())
    torch.cuda.synchronize()
    return gx.cpu().numpy().T, (gm.cpu().numpy() if gm is not None else None)


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_vjp_2048_parity(precision):
    p32, m32, ga, gp, _ = setup(2048, seed=31, masses="random")
    eps = float(np.float32(1 / 64))
    gx, gm = gpu_vjp(p32, m32, eps, ga, gp, precision)
    rx, rm = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                        ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    ex, em = rel_errors(gx, rx), rel_errors(gm, rm)
    print(precision, "grad_pos", ex, "grad_mass", em, "mass scaled max", scaled_max(gm, rm))
    tol = 1e-5 if precision != "plain" else 1e-4
    assert ex["rel_rms"] <= tol and scaled_max(gm, rm) <= tol
    if precision != "plain":
        assert ex["normwise"] <= 1e-6 and em["normwise"] <= 1e-6


@pytest.mark.parametrize("n", [1, 2, 5, 64, 255, 257, 1000, 3001])
def test_vjp_ragged_sizes_and_optional_outputs(n):
    p32, m32, ga, gp, _ = setup(n, seed=40 + n, masses="random")
    eps = 0.02
    rx, rm = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                        ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    gx, gm = gpu_vjp(p32, m32, eps, ga, gp)
    gx2, gm2 = gpu_vjp(p32, m32, eps, ga, gp, with_mass=False)
    np.testing.assert_array_equal(gx, gx2)
    assert gm2 is None
    if n == 1:
        assert np.all(gx == 0) and np.all(gm == 0)
        return
    assert rel_errors(gx, rx)["rel_rms"] <= 1e-5
    assert scaled_max(gm, rm) <= 1e-5
    # No potential cotangent.
    rx0, rm0 = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                          ga.astype(np.float32).astype(np.float64), None)
    gx0, gm0 = gpu_vjp(p32, m32, eps, ga, None)
    assert rel_errors(gx0, rx0)["rel_rms"] <= 1e-5
    assert scaled_max(gm0, rm0) <= 1e-5


@pytest.mark.parametrize("ipl,jtile,nseg", [(1, 64, 3), (2, 128, 1), (4, 256, 5), (8, 512, 2)])
def test_vjp_launch_shapes(ipl, jtile, nseg):
    p32, m32, ga, gp, _ = setup(4000, seed=50)
    eps = 0.01
    rx, rm = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                        ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    gx, gm = gpu_vjp(p32, m32, eps, ga, gp, ipl=ipl, jtile=jtile, nseg=nseg)
    assert rel_errors(gx, rx)["rel_rms"] <= 1e-5 and scaled_max(gm, rm) <= 1e-5


def test_self_pair_adds_nothing_at_tiny_softening():
    # With eps = 1e-3 the j == k term is multiplied by eps^-3 = 1e9: any rounding left in
    # w_kk = m_k g_k - m_k g_k would swamp the true gradient of two distant particles.
    # dL/dm: the j == k term p_k / eps (1e3 |p_k|) is never summed, so only the one real
    # pair's rounding remains (a few u of |p_j| / s + |g_j . d| / s^3, both O(1) here).
    p32 = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, -0.25]], dtype=np.float32)
    m32 = np.array([0.3, 0.7], dtype=np.float32)
    ga = np.array([[0.1, -0.2, 0.3], [0.7, 0.11, -0.5]])
    gp = np.array([0.9, -1.3])
    eps = float(np.float32(1e-3))
    gx, gm = gpu_vjp(p32, m32, eps, ga, gp)
    rx, rm = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                        ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(gx, rx, rtol=1e-5, atol=1e-9)
    u = 2.0 ** -24
    bound = 64 * u * (np.abs(rm) + 1.0)
    assert np.all(np.abs(gm - rm) <= bound), (gm, rm, bound)


def test_vjp_invariants():
    p32, m32, ga, gp, _ = setup(6000, seed=60, masses="random")
    eps = 0.01
    gx, gm = gpu_vjp(p32, m32, eps, ga, gp)
    # translation invariance
    assert np.all(np.abs(gx.sum(0)) < 1e-6 * np.abs(gx).sum(0))
    # degree-1 homogeneity in the masses: sum m dL/dm = sum ga.a + gp.phi
    ra, rp = oracle.force_all(p32.astype(np.float64), m32.astype(np.float64), eps)
    lhs = float((m32.astype(np.float64) * gm).sum())
    rhs = float((ga.astype(np.float32).astype(np.float64) * ra).sum()
                + (gp.astype(np.float32).astype(np.float64) * rp).sum())
    assert abs(lhs - rhs) < 1e-6 * np.abs(m32 * gm).sum()


def test_forcefn_autograd_matches_oracle_vjp():
    n = 3000
    pos, _, mass = ics.plummer(n, seed=70)
    mass = mass * np.random.default_rng(71).uniform(0.5, 1.5, n)
    m32 = mass.astype(np.float32).astype(np.float64)
    eps = float(np.float32(0.01))
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV).requires_grad_(True)
    m = torch.from_numpy(m32).to(DEV).requires_grad_(True)
    rng = np.random.default_rng(72)
    G = rng.standard_normal((3, n))
    P = rng.standard_normal(n)
    acc, pot = autograd.force(x, m, eps)
    loss = (acc * torch.from_numpy(G).to(DEV)).sum() + (pot * torch.from_numpy(P).to(DEV)).sum()
    loss.backward()
    rx, rm = oracle.vjp(pos, m32, eps, G.T.astype(np.float32).astype(np.float64),
                        P.astype(np.float32).astype(np.float64))
    ex = rel_errors(x.grad.cpu().numpy().T, rx)
    em = rel_errors(m.grad.cpu().numpy(), rm)
    print("ForceFn grad_pos", ex, "grad_mass", em)
    assert ex["normwise"] <= 1e-5 and em["normwise"] <= 1e-5


def _rollout_grad(n, seed, eps, dt, steps, target_seed):
    x0, v0, mass = ics.plummer(n, seed=seed)
    m32 = mass.astype(np.float32).astype(np.float64)
    y = ics.perturbed_target(x0, seed=target_seed)
    xt = torch.from_numpy(np.ascontiguousarray(x0.T)).to(DEV).requires_grad_(True)
    vt = torch.from_numpy(np.ascontiguousarray(v0.T)).to(DEV).requires_grad_(True)
    mt = torch.from_numpy(m32).to(DEV).requires_grad_(True)
    yt = torch.from_numpy(np.ascontiguousarray(y.T)).to(DEV)
    xT, vT = autograd.rollout(xt, vt, mt, eps, dt, steps)
    loss = ((xT - yt) ** 2).sum() / n
    loss.backward()
    return (x0, v0, m32, y, float(loss.detach()), xt.grad.cpu().numpy().T, vt.grad.cpu().numpy().T,
            mt.grad.cpu().numpy())


def test_rollout_gradient_small_against_oracle_and_fd():
    n, steps, dt, eps = 64, 32, 1.0 / 256, float(np.float32(0.05))
    x0, v0, m, y, loss, gx, gv, gm = _rollout_grad(n, 80, eps, dt, steps, 81)
    lo, rx, rv, rm = oracle.rollout_loss_grad(x0, v0, m, eps, dt, steps, y)
    # The GPU trajectory carries the FP32 force error (positions off by ~1e-10 against a
    # residual |x - y| ~ 1e-2), so the loss agrees to about 1e-8 relative.
    print("loss", loss, lo, (loss - lo) / lo)
    assert abs(loss - lo) <= 1e-6 * abs(lo)
    for a, b in ((gx, rx), (gv, rv), (gm, rm)):
        assert rel_errors(a, b)["normwise"] <= 1e-5
    # Central FP64 differences of the oracle rollout on 64 seeded coordinates.
    def L(xx, vv, mm):
        xT, _, _, _ = oracle.rollout(xx, vv, mm, eps, dt, steps)
        return float(np.sum((xT - y) ** 2) / n)
    rng = np.random.default_rng(82)
    h = 1e-6
    worst = 0.0
    scale = np.abs(gx).max()
    for _ in range(64):
        k, c = int(rng.integers(n)), int(rng.integers(3))
        xp, xm = x0.copy(), x0.copy()
        xp[k, c] += h
        xm[k, c] -= h
        fd = (L(xp, v0, m) - L(xm, v0, m)) / (2 * h)
        worst = max(worst, abs(fd - gx[k, c]) / scale)
    print("worst FD deviation / max|grad|", worst)
    assert worst < 1e-5


def test_rollout_gradient_adjoint_16384():
    """Workload: N=16384 Plummer, eps=0.01, 32 KDK steps dt=1/256, loss = mean squared
    distance to a perturbed target; GPU adjoint gradient vs the oracle's reverse mode."""
    w = ics.WORKLOADS["adjoint_16384"]
    eps = float(np.float32(w.eps))
    x0, v0, m, y, loss, gx, gv, gm = _rollout_grad(w.n, w.seed, eps, w.dt, w.steps, 5001)
    lo, rx, rv, rm = oracle.rollout_loss_grad(x0, v0, m, eps, w.dt, w.steps, y)
    ex, ev, em = rel_errors(gx, rx), rel_errors(gv, rv), rel_errors(gm, rm)
    print("loss", loss, lo, "grad x0", ex, "v0", ev, "m", em)
    assert abs(loss - lo) <= 1e-6 * abs(lo)
    assert ex["normwise"] <= 1e-4 and ev["normwise"] <= 1e-4 and em["normwise"] <= 1e-4


@pytest.mark.parametrize("centre", ["tile", "system"])
def test_vjp_f64_centres_far_from_origin(centre):
    # FP64 positions offset to (300, 0, -40) and Morton-sorted: the adjoint on positions
    # relative to per-i-tile or per-system FP64 centres matches the oracle VJP on the FP64
    # positions.
    n = 3000
    pos, _, mass = ics.plummer(n, seed=34, velocities=False)
    pos = pos + np.array([300.0, 0.0, -40.0])
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    perm = api.morton_order(x).cpu().numpy().astype(np.int64)
    pos = pos[perm]
    m32 = (mass * np.random.default_rng(35).uniform(0.5, 1.5, n)).astype(np.float32)[perm]
    rng = np.random.default_rng(36)
    ga, gp = rng.standard_normal((n, 3)), rng.standard_normal(n)
    eps = float(np.float32(0.02))
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    g = torch.from_numpy(np.ascontiguousarray(ga.T)).to(DEV)
    gpt = torch.from_numpy(gp).to(DEV)
    gx = torch.empty((3, n), dtype=torch.float64, device=DEV)
    gm = torch.empty(n, dtype=torch.float64, device=DEV)
    _lib.nbody_force_vjp_f64(n, x.data_ptr(), m.data_ptr(), eps, g.data_ptr(), gpt.data_ptr(),
                             gx.data_ptr(), gm.data_ptr(), api.make_opts(centre=centre),
                             api.stream_ptr())
    torch.cuda.synchronize()
    rx, rm = oracle.vjp(pos, m32.astype(np.float64), eps, ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    ex, em = rel_errors(gx.cpu().numpy().T, rx), rel_errors(gm.cpu().numpy(), rm)
    print(centre, "grad_pos", ex, "grad_mass", em)
    assert ex["normwise"] <= 1e-5 and em["normwise"] <= 1e-5


def test_rollout_gradient_with_tile_centres():
    n, steps, dt, eps = 64, 32, 1.0 / 256, float(np.float32(0.05))
    x0, v0, mass = ics.plummer(n, seed=80)
    m32 = mass.astype(np.float32).astype(np.float64)
    y = ics.perturbed_target(x0, seed=81)
    lo, rx, rv, rm = oracle.rollout_loss_grad(x0, v0, m32, eps, dt, steps, y)
    xt = torch.from_numpy(np.ascontiguousarray(x0.T)).to(DEV).requires_grad_(True)
    vt = torch.from_numpy(np.ascontiguousarray(v0.T)).to(DEV).requires_grad_(True)
    mt = torch.from_numpy(m32).to(DEV).requires_grad_(True)
    yt = torch.from_numpy(np.ascontiguousarray(y.T)).to(DEV)
    xT, _ = autograd.rollout(xt, vt, mt, eps, dt, steps, centre="tile")
    loss = ((xT - yt) ** 2).sum() / n
    loss.backward()
    assert abs(float(loss.detach()) - lo) <= 1e-6 * abs(lo)
    for a, b in ((xt.grad.cpu().numpy().T, rx), (vt.grad.cpu().numpy().T, rv),
                 (mt.grad.cpu().numpy(), rm)):
        assert rel_errors(a, b)["normwise"] <= 1e-5


@pytest.mark.parametrize("steps", [0, 1, 4])
def test_rollout_gradient_with_velocity_cotangent(steps):
    # A loss on both final positions and final velocities, L = sum G.x_T + sum H.v_T,
    # through RolloutFn (nbody_leapfrog + nbody_leapfrog_adjoint), against the oracle's
    # reverse mode for the same cotangents (pinned by central differences on the CPU).
    # Zero steps is the identity: the gradients are G and H exactly and dL/dm is zero.
    n, dt, eps = 300, 1.0 / 128, float(np.float32(0.05))
    x0, v0, mass = ics.plummer(n, seed=86)
    m64 = (mass * np.random.default_rng(87).uniform(0.5, 1.5, n)).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(88)
    G, H = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    xt = torch.from_numpy(np.ascontiguousarray(x0.T)).to(DEV).requires_grad_(True)
    vt = torch.from_numpy(np.ascontiguousarray(v0.T)).to(DEV).requires_grad_(True)
    mt = torch.from_numpy(m64).to(DEV).requires_grad_(True)
    xT, vT = autograd.rollout(xt, vt, mt, eps, dt, steps)
    Gt = torch.from_numpy(np.ascontiguousarray(G.T)).to(DEV)
    Ht = torch.from_numpy(np.ascontiguousarray(H.T)).to(DEV)
    ((xT * Gt).sum() + (vT * Ht).sum()).backward()
    gx, gv, gm = xt.grad.cpu().numpy().T, vt.grad.cpu().numpy().T, mt.grad.cpu().numpy()
    rx, rv, rm = oracle.rollout_vjp(x0, v0, m64, eps, dt, steps, G, H)
    if steps == 0:
        assert np.array_equal(gx, G) and np.array_equal(gv, H) and not gm.any()
        return
    ex, ev, em = rel_errors(gx, rx), rel_errors(gv, rv), rel_errors(gm, rm)
    print(steps, "grad x0", ex, "v0", ev, "m", em)
    assert ex["normwise"] <= 1e-5 and ev["normwise"] <= 1e-5 and em["normwise"] <= 1e-5
