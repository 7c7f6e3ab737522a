"""GPU ragged batches (persistent work-queue kernel) against the FP64 oracle run
system by system, plus graph replay of the batched leapfrog."""
import numpy as np
import pytest
import torch

import bounds
import oracle
from paper_astro_ph_0703100_amd import api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def ragged(sizes, seed, eps_list=None):
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    pos = np.zeros((total, 3))
    vel = np.zeros((total, 3))
    mass = np.zeros(total)
    for k, n in enumerate(sizes):
        if n == 0:
            continue
        p, v, m = ics.plummer(int(n), seed=seed + k)
        m = m * np.random.default_rng(seed + 100 + k).uniform(0.5, 1.5, n)
        s, e = offsets[k], offsets[k + 1]
        pos[s:e], vel[s:e], mass[s:e] = p + 3.0 * k, v, m  # systems apart; they do not interact
    eps = np.array(eps_list if eps_list is not None else [0.01] * len(sizes), dtype=np.float32)
    return offsets, pos, vel, mass.astype(np.float32), eps


def oracle_batch(offsets, pos, m32, eps, systems=None):
    out = {}
    for k in systems if systems is not None else range(len(offsets) - 1):
        s, e = offsets[k], offsets[k + 1]
        if e > s:
            out[k] = oracle.force_all(pos[s:e], m32[s:e].astype(np.float64), float(eps[k]))
    return out


def check_system_bounds(acc, pot, ra, rp, x, m32, eps, precision):
    """Per-particle bounds of tests/bounds.py for one system (acc/pot: its rows)."""
    n = x.shape[0]
    absa, absp = oracle.force_abs_sampled(x, m32.astype(np.float64), eps, np.arange(n))
    wa = bounds.check_acc(acc, ra, absa, precision, n)
    wp = bounds.check_pot(pot, rp, absp, precision, n) if pot is not None else 0.0
    return wa, wp


SIZES = [0, 1, 2, 255, 256, 257, 1000, 3001, 1, 4097, 64, 0, 777]
EPS = [0.01, 0.02, 0.005, 0.03, 0.01, 0.01, 0.015, 0.01, 0.02, 0.008, 0.05, 0.01, 0.01]


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
@pytest.mark.parametrize("ipl,jtile", [(0, 0), (1, 64), (4, 256), (8, 512)])
def test_batched_force_matches_oracle_per_system(precision, ipl, jtile):
    offsets, pos, _, m32, eps = ragged(SIZES, seed=200, eps_list=EPS)
    x32 = pos.astype(np.float32)
    plan = api.BatchPlan(offsets, precision=precision, ipl=ipl, jtile=jtile)
    info = plan.info()
    assert info["nsys"] == len(SIZES) and info["total"] == offsets[-1]
    p = torch.from_numpy(np.ascontiguousarray(x32.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    acc, pot = plan.force(p, m, e)
    torch.cuda.synchronize()
    acc, pot = acc.cpu().numpy().T, pot.cpu().numpy()
    ref = oracle_batch(offsets, x32.astype(np.float64), m32, eps)
    tol = 1e-6 if precision != "plain" else 1e-5
    for k, (ra, rp) in ref.items():
        s, t = offsets[k], offsets[k + 1]
        if t - s == 1:
            assert np.all(acc[s:t] == 0) and np.all(pot[s:t] == 0)
            continue
        ea, ep = rel_errors(acc[s:t], ra), rel_errors(pot[s:t], rp)
        assert ea["rel_rms"] <= tol, (k, t - s, ea)
        assert ep["rel_rms"] <= tol, (k, t - s, ep)
        check_system_bounds(acc[s:t], pot[s:t], ra, rp, x32[s:t].astype(np.float64), m32[s:t],
                            float(eps[k]), precision)
    plan.close()


def test_batched_is_deterministic_and_f64_path_matches():
    offsets, pos, vel, m32, eps = ragged([5000, 300, 12000, 1, 2048], seed=300)
    plan = api.BatchPlan(offsets)
    x64 = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    a1, p1 = plan.force_f64(x64, m, e)
    a2, p2 = plan.force_f64(x64, m, e)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    ref = oracle_batch(offsets, pos, m32, eps)
    a1 = a1.cpu().numpy().T
    for k, (ra, rp) in ref.items():
        s, t = offsets[k], offsets[k + 1]
        if t - s > 1:
            assert rel_errors(a1[s:t], ra)["rel_rms"] <= 1e-6, k
    plan.close()


@pytest.mark.parametrize("precision,ipl,jtile", [("comp", 1, 64), ("fp64red", 2, 256),
                                                  ("plain", 1, 128)])
def test_batched_equals_single_system_calls_bitwise(precision, ipl, jtile):
    # A plan splits system k into i-tiles and S_k j-segments of about 4096 j's; the
    # single-system entry point at the same IPL, j-tile and S_k runs the same blocks and
    # the same fixed-order reduction, so every system's result is the same bits.
    sizes = [5000, 300, 9000, 0, 1, 4097, 64]
    offsets, pos, _, m32, eps = ragged(sizes, seed=400, eps_list=[0.01, 0.02, 0.005, 0.01,
                                                                  0.01, 0.03, 0.01])
    plan = api.BatchPlan(offsets, precision=precision, ipl=ipl, jtile=jtile)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    acc, pot = plan.force(p, m, torch.from_numpy(eps).to(DEV))
    torch.cuda.synchronize()
    per_seg_tiles = max(1, 4096 // jtile)
    for k, n in enumerate(sizes):
        if n < 2:
            continue
        s, t = int(offsets[k]), int(offsets[k + 1])
        jtiles = -(-n // jtile)
        segs = -(-jtiles // per_seg_tiles)
        per = -(-jtiles // segs)
        segs = -(-jtiles // per)
        a1, p1 = api.force(p[:, s:t].contiguous(), m[s:t].contiguous(), float(eps[k]),
                           precision=precision, ipl=ipl, jtile=jtile, nseg=segs)
        torch.cuda.synchronize()
        assert torch.equal(acc[:, s:t], a1), (k, n)
        assert torch.equal(pot[s:t], p1), (k, n)
    plan.close()


def test_batched_graph_replay_is_bitwise_eager():
    offsets, pos, vel, m32, eps = ragged([3000, 1000, 257, 6000], seed=400)
    plan = api.BatchPlan(offsets)
    x0 = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    v0 = torch.from_numpy(np.ascontiguousarray(vel.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    a0, _ = plan.leapfrog(x0.clone(), v0.clone(), m, e, 1 / 512, 0)
    xe, ve, ae = x0.clone(), v0.clone(), a0.clone()
    plan.leapfrog(xe, ve, m, e, 1 / 512, 4, acc=ae, init=False)
    torch.cuda.synchronize()
    xg, vg, ag = x0.clone(), v0.clone(), a0.clone()
    g = plan.graph(xg, vg, m, e, 1 / 512, 4, ag)
    for rep in range(3):
        xg.copy_(x0)
        vg.copy_(v0)
        ag.copy_(a0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(vg, ve) and torch.equal(ag, ae), rep
    g.close()
    plan.close()


def test_clusters_2048_graph_leapfrog():
    """Workload: 2048 independent Plummer clusters, N_k log-uniform in [256, 16384],
    eps = 0.01, masses 1/N_k, 16 graph-captured KDK steps dt = 1/512 (one persistent
    launch per force evaluation).  16 seeded systems, including the smallest and
    largest, are checked against the oracle at step 0 and at the GPU's step-16
    positions."""
    w = ics.WORKLOADS["clusters_2048"]
    b = ics.cluster_batch(w.n, seed=w.seed, eps=w.eps)
    m32 = b.mass.astype(np.float32)
    eps = b.eps.astype(np.float32)
    plan = api.BatchPlan(b.offsets)
    print("plan", plan.info())
    x = torch.from_numpy(np.ascontiguousarray(b.pos.T)).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(b.vel.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    acc0, pot0 = plan.leapfrog(x, v, m, e, w.dt, 0, with_pot=True)
    sizes = b.sizes
    rng = np.random.default_rng(w.seed + 1000)
    pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] +
                      list(rng.choice(b.nsys, size=14, replace=False))))
    assert min(sizes[k] for k in pick) < 300  # a smallest-cluster system is among them

    def check(a, p, xs, label):
        # Per system: acceleration and potential relative RMS <= 1e-6 against the oracle
        # on the FP64 positions, and every particle inside the rounding bound against the
        # oracle on the FP32 inputs the kernel sees, fp32(x - c) with c the FP64 mean
        # position of the system (the bound covers the pair arithmetic, not the input
        # rounding).  Clusters of a few hundred particles have m_i / eps of the order of
        # |phi_i|: no self term may leak into phi.
        for k, (ra, rp) in oracle_batch(b.offsets, xs, m32, eps, pick).items():
            s, t = b.offsets[k], b.offsets[k + 1]
            ea, ep = rel_errors(a[s:t], ra), rel_errors(p[s:t], rp)
            assert ea["rel_rms"] <= 1e-6, (label, k, t - s, ea)
            assert ep["rel_rms"] <= 1e-6, (label, k, t - s, ep)
            xk = xs[s:t]
            x32 = (xk - xk.mean(axis=0)).astype(np.float32).astype(np.float64)
            ra32, rp32 = oracle.force_all(x32, m32[s:t].astype(np.float64), float(eps[k]))
            check_system_bounds(a[s:t], p[s:t], ra32, rp32, x32, m32[s:t], float(eps[k]),
                                "comp")

    check(acc0.cpu().numpy().T, pot0.cpu().numpy(), b.pos, "step 0")
    pot = torch.empty_like(pot0)
    g = plan.graph(x, v, m, e, w.dt, w.steps, acc0, pot)
    g.launch()
    torch.cuda.synchronize()
    check(acc0.cpu().numpy().T, pot.cpu().numpy(), x.cpu().numpy().T, "step 16")
    g.close()
    plan.close()
