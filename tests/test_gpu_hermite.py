"""GPU fourth-order Hermite integration (nbody_hermite, its graph) against the oracle.

The GPU state is FP64 and each step evaluates forces and jerks in FP32 pair
arithmetic relative to the system centres, so the trajectory differs from the FP64
oracle's by what the force error does over the run: with Delta a the largest
acceleration error of one evaluation (measured at the initial state against the
oracle) and T the run time, positions may differ by about T^2 Delta a and velocities
by T Delta a, times a growth factor for the divergence of nearby orbits (10 here).
A wrong predictor or corrector coefficient gives errors of order dt^3 |snap| per step,
far above that bound on the smooth, strongly softened system used first.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import _lib, api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def state(n, seed, offset=(0.0, 0.0, 0.0)):
    x, v, m = ics.plummer(n, seed=seed)
    x = x + np.asarray(offset)
    m32 = m.astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV)
    return x, v, m32, t(x), t(v), torch.from_numpy(m32).to(DEV)


def force_error(xd, vd, md, x, v, m64, eps, precision):
    """Largest |Delta a| of one GPU evaluation at the given state (vs the oracle)."""
    acc, _, _ = api.force_jerk(xd, vd, md, eps, precision=precision)
    ref, _, _ = oracle.force_jerk(x, v, m64, eps)
    return float(np.sqrt(((acc.cpu().numpy().T - ref) ** 2).sum(1)).max())


@pytest.mark.parametrize("precision", ["comp", "fp64red"])
@pytest.mark.parametrize("n,eps,dt,steps,seed", [(256, 0.25, 1.0 / 128, 32, 70),
                                                 (2048, 0.01, 1.0 / 256, 16, 71)])
def test_hermite_matches_oracle(precision, n, eps, dt, steps, seed):
    eps = float(np.float32(eps))
    x, v, m32, xd, vd, md = state(n, seed, offset=(3.0, -1.0, 2.0))
    m64 = m32.astype(np.float64)
    da = force_error(xd, vd, md, x, v, m64, eps, precision)
    acc, jerk = api.hermite(xd, vd, md, eps, dt, steps, precision=precision)
    torch.cuda.synchronize()
    xo, vo, ao, jo = oracle.hermite(x, v, m64, eps, dt, steps)
    dx = np.abs(xd.cpu().numpy().T - xo).max()
    dv = np.abs(vd.cpu().numpy().T - vo).max()
    ea = rel_errors(acc.cpu().numpy().T, ao)
    ej = rel_errors(jerk.cpu().numpy().T, jo)
    T = dt * steps
    print(precision, n, "dx %.2e (bound %.2e) dv %.2e (bound %.2e) acc %s jerk %s"
          % (dx, 10 * T * T * da, dv, 10 * T * da, ea, ej))
    assert dx <= 10 * T * T * da and dv <= 10 * T * da
    assert ea["rel_rms"] < 1e-6
    assert ej["normwise"] < 1e-5


def test_free_particle_and_continuation():
    # One particle: a = j = 0, the predictor and corrector reduce to x += v dt.
    x = torch.tensor([[1.0], [2.0], [3.0]], dtype=torch.float64, device=DEV)
    v = torch.tensor([[0.5], [-0.25], [2.0]], dtype=torch.float64, device=DEV)
    m = torch.ones(1, dtype=torch.float32, device=DEV)
    acc, jerk = api.hermite(x, v, m, 0.1, 0.125, 8)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x.cpu().numpy().ravel(), [1.5, 1.75, 5.0])
    assert torch.all(acc == 0) and torch.all(jerk == 0)
    # Two calls of 3 steps (the second continuing from the returned a, j) equal one of 6.
    n, dt, eps = 1500, 1.0 / 128, 0.02
    _, _, _, xa, va, md = state(n, 73)
    xb, vb = xa.clone(), va.clone()
    a1, j1 = api.hermite(xa, va, md, eps, dt, 6)
    a2, j2 = api.hermite(xb, vb, md, eps, dt, 3)
    a2, j2 = api.hermite(xb, vb, md, eps, dt, 3, acc=a2, jerk=j2, init=False)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert torch.equal(a1, a2) and torch.equal(j1, j2)


def test_graph_replays_equal_eager():
    n, dt, eps, steps = 3000, 1.0 / 256, 0.01, 5
    _, _, _, x0, v0, md = state(n, 75)
    xe, ve = x0.clone(), v0.clone()
    ae, je = api.hermite(xe, ve, md, eps, dt, steps)
    xg, vg = x0.clone(), v0.clone()
    ag, jg = api.hermite(xg, vg, md, eps, dt, 0)  # a, j at the start
    g = api.HermiteGraph(xg, vg, md, eps, dt, 1, ag, jg)
    for t in range(steps):
        g.launch()
        torch.cuda.synchronize()
        _ = (xg.sum() + ag.sum()).item()  # unrelated eager work between replays
    g.close()
    assert torch.equal(xg, xe) and torch.equal(vg, ve)
    assert torch.equal(ag, ae) and torch.equal(jg, je)


def test_hermite_with_tile_centres_and_bad_arguments():
    # Morton-sorted system far from the origin: per-i-tile centres of position and
    # velocity; the trajectory matches the oracle like the system-centre path.
    n, dt, steps = 2000, 1.0 / 256, 8
    eps = float(np.float32(0.02))
    x, v, m = ics.plummer(n, seed=79)
    x = x + np.array([500.0, 20.0, -30.0])
    v = v + np.array([-10.0, 5.0, 0.0])
    xt = torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)
    perm = api.morton_order(xt).cpu().numpy().astype(np.int64)
    x, v, m32 = x[perm], v[perm], m[perm].astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV)
    xd, vd, md = t(x), t(v), torch.from_numpy(m32).to(DEV)
    m64 = m32.astype(np.float64)
    da = force_error(xd, vd, md, x, v, m64, eps, "comp")
    acc, jerk = api.hermite(xd, vd, md, eps, dt, steps, centre="tile")
    torch.cuda.synchronize()
    xo, vo, ao, jo = oracle.hermite(x, v, m64, eps, dt, steps)
    T = dt * steps
    dx = np.abs(xd.cpu().numpy().T - xo).max()
    dv = np.abs(vd.cpu().numpy().T - vo).max()
    print("tile centres: dx %.2e dv %.2e (system-centre force error %.2e)" % (dx, dv, da))
    assert dx <= 10 * T * T * da and dv <= 10 * T * da
    assert rel_errors(acc.cpu().numpy().T, ao)["rel_rms"] < 1e-6
    acc = torch.empty_like(xd)
    jerk = torch.empty_like(xd)
    assert _lib.nbody_hermite(n, xd.data_ptr(), vd.data_ptr(), md.data_ptr(), 0.01, float("nan"), 2,
                              acc.data_ptr(), jerk.data_ptr(), 0, None, None,
                              check=False) == _lib.NBODY_EINVAL


def test_paper_scale_hermite_graph_steps():
    """The benchmark's configuration: N = 131072, one captured Hermite step replayed
    (dt = 1/256).  The replays equal eager steps bitwise, and after them the returned
    acceleration and jerk (those of the last predicted state) match the oracle at that
    state on 1024 seeded particles."""
    w = ics.WORKLOADS["jerk_131072"]
    x, v, m32, xd, vd, md = state(w.n, w.seed)
    eps = float(np.float32(w.eps))
    steps = 2
    xe, ve = xd.clone(), vd.clone()
    ae, je = api.hermite(xe, ve, md, eps, w.dt, steps)
    xg, vg = xd.clone(), vd.clone()
    ag, jg = api.hermite(xg, vg, md, eps, w.dt, 0)
    g = api.HermiteGraph(xg, vg, md, eps, w.dt, 1, ag, jg)
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    g.close()
    assert torch.equal(xg, xe) and torch.equal(vg, ve)
    assert torch.equal(ag, ae) and torch.equal(jg, je)
    # Rebuild the last predicted state from the state before the last step.
    xb, vb = xd.clone(), vd.clone()
    ab, jb = api.hermite(xb, vb, md, eps, w.dt, steps - 1)
    torch.cuda.synchronize()
    dt = w.dt
    xp = (xb + vb * dt + ab * dt * dt / 2 + jb * dt ** 3 / 6).cpu().numpy().T
    vp = (vb + ab * dt + jb * dt * dt / 2).cpu().numpy().T
    idx = ics.sample_indices(w.n, 1024, seed=w.seed + 1000)
    ra, rj, _ = oracle.force_jerk(xp, vp, m32.astype(np.float64), eps, idx=idx)
    ea = rel_errors(ae.cpu().numpy().T[idx], ra)
    ej = rel_errors(je.cpu().numpy().T[idx], rj)
    print("acc", ea, "jerk", ej)
    assert ea["rel_rms"] <= 1e-6
    assert ej["normwise"] <= 1e-5
