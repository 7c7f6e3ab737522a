"""Split engine (each i-particle's j-range spread over lanes of a wavefront, FP64
cross-lane sums, one launch) against the FP64 oracle.

Same tolerances as the grid engine: relative RMS <= 1e-6 (compensated, FP64-reduced)
or 1e-5 (plain), and the per-component rounding bound of tests/bounds.py on every
particle.  A lane's FP32 block is its share of one tile, JT / jlanes <= 128 terms, so
the bound's block term is (JT / jlanes - 1) u for the blocked modes; plain FP32 sums a
lane's whole share, then the jlanes shares in FP32 (fewer than n + 64 additions).
Shapes cover every jlanes, both ipl, every j-tile, ragged n (last block and last tile
partly empty), n below one block, and the self pair in every tile position.
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

SHAPES = [(1, 8, 256), (1, 8, 1024), (1, 16, 512), (1, 32, 256), (1, 32, 1024), (1, 32, 2048),
          (1, 64, 256), (1, 64, 512), (1, 64, 2048), (2, 8, 512), (2, 16, 256), (2, 32, 512),
          (2, 64, 1024), (2, 64, 2048)]


def split_adds(precision, n, jlanes, jtile):
    if precision == "plain":
        return n + 64
    return min(128, jtile // jlanes) - 1


def to_dev(pos, mass):
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    return (torch.from_numpy(p32).to(DEV), torch.from_numpy(m32).to(DEV),
            p32.T.astype(np.float64), m32.astype(np.float64))


def check(acc, pot, ra, rp, x64, m64, eps, precision, n, jl, jt):
    absa, absp = oracle.force_abs_sampled(x64, m64, eps, np.arange(n))
    a = split_adds(precision, n, jl, jt)
    ratio_a = np.abs(acc - ra) / (U * np.maximum(absa, 1e-300))
    ratio_p = np.abs(pot - rp) / (U * np.maximum(absp, 1e-300))
    assert ratio_a.max() <= bounds.C_ACC + a, (precision, float(ratio_a.max()))
    assert ratio_p.max() <= bounds.C_POT + a, (precision, float(ratio_p.max()))
    return float(ratio_a.max()), float(ratio_p.max())


@pytest.mark.parametrize("ipl,jl,jt", SHAPES)
def test_split_shapes_match_oracle(ipl, jl, jt):
    n = 3001
    pos, _, mass = ics.plummer(n, seed=500 + jl, velocities=False)
    mass = mass * np.random.default_rng(jl + jt).uniform(0.5, 1.5, n)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    for precision in ("comp", "fp64red", "plain"):
        acc, pot = api.force(p, m, eps, precision=precision, ipl=ipl, jtile=jt, jlanes=jl)
        acc2, pot2 = api.force(p, m, eps, precision=precision, ipl=ipl, jtile=jt, jlanes=jl)
        torch.cuda.synchronize()
        assert torch.equal(acc, acc2) and torch.equal(pot, pot2)  # reproducible
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
        wa, wp = check(acc, pot, ra, rp, x64, m64, eps, precision, n, jl, jt)
        print(ipl, jl, jt, precision, "acc", ea, "pot", ep, "bound ratios %.1f %.1f" % (wa, wp))
        assert ea["rel_rms"] <= TOL[precision], (precision, ea)
        assert ep["rel_rms"] <= TOL[precision], (precision, ep)


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 255, 1023, 1025, 2048, 4097])
def test_split_ragged_sizes(n):
    pos, _, mass = ics.plummer(n, seed=900 + n, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.02
    ra, rp = oracle.force_all(x64, m64, eps)
    for ipl, jl, jt in [(1, 64, 256), (2, 8, 1024), (1, 16, 512)]:
        acc, pot = api.force(p, m, eps, ipl=ipl, jtile=jt, jlanes=jl)
        torch.cuda.synchronize()
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        if n == 1:
            assert np.all(acc == 0) and np.all(pot == 0)
            continue
        assert rel_errors(acc, ra)["rel_rms"] <= 1e-6
        check(acc, pot, ra, rp, x64, m64, eps, "comp", n, jl, jt)


def test_split_self_potential_and_no_potential():
    n = 777
    pos, _, mass = ics.plummer(n, seed=8, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = 0.01
    ra, rp = oracle.force_all(x64, m64, eps)
    acc, pot = api.force(p, m, eps, self_pot=True, jlanes=32, jtile=512)
    acc0, pot0 = api.force(p, m, eps, with_pot=False, jlanes=32, jtile=512)
    acc1, _ = api.force(p, m, eps, jlanes=32, jtile=512)
    torch.cuda.synchronize()
    assert pot0 is None
    assert torch.equal(acc0, acc1)  # the potential-free kernel sums the same terms
    pot = pot.cpu().numpy()
    assert rel_errors(pot, rp - m64 / np.float64(np.float32(eps)))["rel_rms"] <= 1e-6


def test_plummer_2048_default_shape():
    """Workload: N = 2048 Plummer sphere, eps = 1/64, every mode, default launch shape (the
    tuned shape for this size), all N^2 pairs against the oracle."""
    w = ics.WORKLOADS["plummer_2048"]
    pos, _, mass = ics.plummer(w.n, seed=w.seed, velocities=False)
    p, m, x64, m64 = to_dev(pos, mass)
    eps = float(np.float32(w.eps))
    ra, rp = oracle.force_all(x64, m64, eps)
    ipl, jt, _, jl, _ = _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, w.n)
    for precision in ("comp", "fp64red", "plain"):
        acc, pot = api.force(p, m, eps, precision=precision)
        torch.cuda.synchronize()
        acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
        ea, ep = rel_errors(acc, ra), rel_errors(pot, rp)
        print(precision, (ipl, jt, jl), "acc", ea, "pot", ep)
        assert ea["rel_rms"] <= TOL[precision] and ep["rel_rms"] <= TOL[precision]


@pytest.mark.parametrize("ipl,jl,jt", [(1, 8, 256), (1, 16, 512), (2, 32, 512), (1, 64, 256)])
def test_split_vjp_matches_oracle(ipl, jl, jt):
    n = 2500
    pos, _, mass = ics.plummer(n, seed=77, velocities=False)
    mass = mass * np.random.default_rng(78).uniform(0.5, 1.5, n)
    p32, m32 = pos.astype(np.float32), mass.astype(np.float32)
    rng = np.random.default_rng(79)
    ga, gp = rng.standard_normal((n, 3)), rng.standard_normal(n)
    eps = 0.01
    rx, rm = oracle.vjp(p32.astype(np.float64), m32.astype(np.float64), eps,
                        ga.astype(np.float32).astype(np.float64),
                        gp.astype(np.float32).astype(np.float64))
    p = torch.from_numpy(np.ascontiguousarray(p32.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    g = torch.from_numpy(np.ascontiguousarray(ga.T)).to(DEV)
    gpt = torch.from_numpy(gp).to(DEV)
    for precision in ("comp", "fp64red", "plain"):
        gx = torch.empty((3, n), dtype=torch.float64, device=DEV)
        gm = torch.empty(n, dtype=torch.float64, device=DEV)
        opts = api.make_opts(precision=precision, ipl=ipl, jtile=jt, jlanes=jl)
        _lib.nbody_force_vjp(n, p.data_ptr(), m.data_ptr(), eps, g.data_ptr(), gpt.data_ptr(),
                             gx.data_ptr(), gm.data_ptr(), opts, api.stream_ptr())
        torch.cuda.synchronize()
        ex = rel_errors(gx.cpu().numpy().T, rx)
        em = rel_errors(gm.cpu().numpy(), rm)
        scaled = float(np.abs(gm.cpu().numpy() - rm).max() / np.sqrt(np.mean(rm ** 2)))
        print(ipl, jl, jt, precision, "grad_pos", ex, "grad_mass", em, "scaled max %.2e" % scaled)
        tol = 1e-5 if precision != "plain" else 1e-4
        assert ex["rel_rms"] <= tol and scaled <= tol
        if precision != "plain":
            assert ex["normwise"] <= 1e-6 and em["normwise"] <= 1e-6


def test_split_leapfrog_matches_grid_engine_rollout():
    """Two KDK steps with the split engine (FP64 state, system centre, kick fused into
    the output stage) against the same steps with the grid engine: both within the
    force tolerance of the oracle at the final positions."""
    n = 4096
    pos, vel, mass = ics.plummer(n, seed=55)
    m32 = mass.astype(np.float32)
    eps, dt = 0.01, 1.0 / 256
    m = torch.from_numpy(m32).to(DEV)
    out = {}
    for name, kw in (("split", dict(jlanes=16, jtile=512)), ("grid", dict(jlanes=1))):
        x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
        v = torch.from_numpy(np.ascontiguousarray(vel.T)).to(DEV)
        acc, pot, _ = api.leapfrog(x, v, m, eps, dt, 2, with_pot=True, **kw)
        torch.cuda.synchronize()
        out[name] = (x.cpu().numpy().T, v.cpu().numpy().T, acc.cpu().numpy().T, pot.cpu().numpy())
    xs, _, acc, pot = out["split"]
    ra, rp = oracle.force_all(xs, m32.astype(np.float64), eps)
    assert rel_errors(acc, ra)["rel_rms"] <= 1e-6
    assert rel_errors(pot, rp)["rel_rms"] <= 1e-6
    # the two engines round differently but follow the same trajectory closely
    assert np.abs(out["split"][0] - out["grid"][0]).max() < 1e-9


def test_split_rejected_where_not_built():
    """Entry points without a split-engine kernel refuse jlanes > 1 before enqueuing."""
    n = 1000
    pos, vel, mass = ics.plummer(n, seed=5)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    with pytest.raises(_lib.NBodyError) as e:
        api.force_ij(p, p, m, 0.01, jlanes=16)
    assert e.value.status == _lib.NBODY_EUNSUPPORTED
    with pytest.raises(_lib.NBodyError) as e:
        api.force(p, m, 0.01, jlanes=16, jtile=64)
    assert e.value.status == _lib.NBODY_EINVAL


def test_split_leapfrog_graph_replays_match_eager_steps():
    """Captured KDK steps with the split engine (the graph owns its scratch): every replay,
    with eager work between them, gives bitwise the eager steps' state."""
    n, steps, dt, eps = 2500, 3, 1.0 / 256, 0.01
    pos, vel, mass = ics.plummer(n, seed=61)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    shape = dict(ipl=1, jtile=1024, jlanes=32)

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


@pytest.mark.parametrize("steps", [1, 4])
def test_split_leapfrog_adjoint_matches_oracle(steps):
    """nbody_leapfrog_adjoint with the split engine for both the forward rebuild and the
    adjoint evaluations, against the oracle's reverse mode for cotangents on x_T and v_T."""
    n, dt, eps = 1500, 1.0 / 128, float(np.float32(0.05))
    x0, v0, mass = ics.plummer(n, seed=62)
    m32 = (mass * np.random.default_rng(63).uniform(0.5, 1.5, n)).astype(np.float32)
    m64 = m32.astype(np.float64)
    rng = np.random.default_rng(64)
    G, H = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    shape = dict(ipl=1, jtile=512, jlanes=16)
    x = torch.from_numpy(np.ascontiguousarray(x0.T)).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(v0.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    _, _, traj = api.leapfrog(x, v, m, eps, dt, steps, keep_trajectory=True, **shape)
    xbar = torch.from_numpy(np.ascontiguousarray(G.T)).to(DEV)
    vbar = torch.from_numpy(np.ascontiguousarray(H.T)).to(DEV)
    mbar = torch.zeros(n, dtype=torch.float64, device=DEV)
    _lib.nbody_leapfrog_adjoint(n, traj.data_ptr(), m.data_ptr(), eps, dt, steps,
                                xbar.data_ptr(), vbar.data_ptr(), mbar.data_ptr(),
                                api.make_opts(**shape), api.stream_ptr())
    torch.cuda.synchronize()
    rx, rv, rm = oracle.rollout_vjp(x0, v0, m64, eps, dt, steps, G, H)
    ex = rel_errors(xbar.cpu().numpy().T, rx)
    ev = rel_errors(vbar.cpu().numpy().T, rv)
    em = rel_errors(mbar.cpu().numpy(), rm)
    print(steps, "grad x0", ex, "v0", ev, "m", em)
    assert ex["normwise"] <= 1e-5 and ev["normwise"] <= 1e-5 and em["normwise"] <= 1e-5
