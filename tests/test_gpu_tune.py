"""The autotuner on the GPU: every launch shape of a sweep (grid and split engines) is
timed and checked against an FP64-reduced run at the built-in shape, the fastest
admitted shape is what the table then serves, a shape whose result misses the gate is
never admitted, and the admitted winners agree with the FP64 oracle to the stated
tolerances (the tuner's own gate compares the GPU with itself)."""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import _lib, api, ics, tune
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(autouse=True)
def committed_table():
    yield
    _lib.nbody_tune_reset()
    _lib.nbody_tune_load(_lib.TUNING_PATH)


def check_sweep(best, rows, n, kernel):
    assert len(rows) == len(tune.shapes(n, kernel))
    assert all(r["ok"] for r in rows), [r for r in rows if not r["ok"]][:3]
    assert best["ms"] == min(r["ms"] for r in rows)


def shape_of(best):
    return {k: best[k] for k in ("ipl", "jtile", "nseg", "jlanes")}


def test_force_sweep_admits_every_shape_and_the_table_serves_the_best():
    n, eps = 3001, 0.02
    best, rows = tune.tune_force(n, 7, eps, "comp", reps=1)
    check_sweep(best, rows, n, "force")
    assert any(r["jlanes"] > 1 for r in rows) and any(r["jlanes"] == 1 for r in rows)
    _lib.nbody_tune_set(_lib.KERNELS["force"], _lib.PRECISIONS["comp"], n, best["ipl"],
                        best["jtile"], best["nseg"], best["jlanes"])
    assert _lib.nbody_tune_get(_lib.KERNELS["force"], _lib.PRECISIONS["comp"], n) == \
        (best["ipl"], best["jtile"], best["nseg"], best["jlanes"], 0)
    pos, _, mass = ics.plummer(n, seed=7)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    a_table, p_table = api.force(p, m, eps)
    a_shape, p_shape = api.force(p, m, eps, **shape_of(best))
    torch.cuda.synchronize()
    assert torch.equal(a_table, a_shape) and torch.equal(p_table, p_shape)
    # the winner against the oracle
    x64 = pos.astype(np.float32).astype(np.float64)
    m64 = mass.astype(np.float32).astype(np.float64)
    ra, rp = oracle.force_all(x64, m64, eps)
    assert rel_errors(a_table.cpu().numpy().T, ra)["rel_rms"] <= 1e-6
    assert rel_errors(p_table.cpu().numpy(), rp)["rel_rms"] <= 1e-6


def test_force_sweep_winners_match_oracle_at_several_sizes():
    """The fastest admitted shape of each mode at sizes where the split engine and the grid
    engine compete, checked against the oracle (all N^2 pairs)."""
    for n, prec in ((2048, "comp"), (2048, "plain"), (8192, "fp64red")):
        best, rows = tune.tune_force(n, 20 + n, 0.01, prec, reps=1)
        pos, _, mass = ics.plummer(n, seed=20 + n)
        p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
        m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
        acc, pot = api.force(p, m, 0.01, precision=prec, **shape_of(best))
        torch.cuda.synchronize()
        ra, rp = oracle.force_all(pos.astype(np.float32).astype(np.float64),
                                  mass.astype(np.float32).astype(np.float64), 0.01)
        tol = 1e-6 if prec != "plain" else 1e-5
        ea = rel_errors(acc.cpu().numpy().T, ra)
        ep = rel_errors(pot.cpu().numpy(), rp)
        print(n, prec, shape_of(best), "%.4f ms" % best["ms"], ea, ep)
        assert ea["rel_rms"] <= tol and ep["rel_rms"] <= tol


def test_jerk_and_vjp_sweeps():
    n = 1500
    best, rows = tune.tune_jerk(n, 8, 0.03, "comp", reps=1)
    assert len(rows) == sum(1 for _ in tune.IPLS for jt in tune.JTILES for s in tune.SEGS
                            if s <= (n + jt - 1) // jt)
    assert all(r["ok"] for r in rows) and best["ms"] == min(r["ms"] for r in rows)
    # the jerk winner against the oracle
    pos, vel, mass = ics.plummer(n, seed=8)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(vel.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    acc, jerk, _ = api.force_jerk(p, v, m, 0.03, ipl=best["ipl"], jtile=best["jtile"],
                                  nseg=best["nseg"])
    torch.cuda.synchronize()
    f = lambda a: a.astype(np.float32).astype(np.float64)
    ra, rj, _ = oracle.force_jerk(f(pos), f(vel), f(mass), 0.03)
    assert rel_errors(acc.cpu().numpy().T, ra)["rel_rms"] <= 1e-6
    assert rel_errors(jerk.cpu().numpy().T, rj)["normwise"] <= 1e-5

    best, rows = tune.tune_vjp(n, 9, 0.03, "comp", reps=1)
    check_sweep(best, rows, n, "vjp")
    # the adjoint winner against the oracle (the sweep's cotangent: dL/da only)
    pos, _, mass = ics.plummer(n, seed=9)
    ga = np.random.default_rng(10).standard_normal((3, n))
    rx, _ = oracle.vjp(f(pos), f(mass), 0.03, f(ga.T), None)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    g = torch.from_numpy(ga).to(DEV)
    gx = torch.empty((3, n), dtype=torch.float64, device=DEV)
    opts = api.make_opts(**shape_of(best))
    _lib.nbody_force_vjp(n, p.data_ptr(), m.data_ptr(), 0.03, g.data_ptr(), None,
                         gx.data_ptr(), None, opts, api.stream_ptr())
    torch.cuda.synchronize()
    assert rel_errors(gx.cpu().numpy().T, rx)["normwise"] <= 1e-6


def test_batched_sweep():
    best, rows = tune.tune_batched(6, 10, 0.01, "comp", reps=1)
    assert len(rows) == len(tune.IPLS) * len(tune.JTILES)
    assert all(r["ok"] for r in rows)
    assert best["ms"] == min(r["ms"] for r in rows)


def test_gate_rejects_results_that_miss_it(monkeypatch):
    # Plain FP32 accumulation cannot meet a 1e-12 gate: no shape may be admitted.
    monkeypatch.setitem(tune.GATE, "plain", 1e-12)
    best, rows = tune.tune_force(1024, 11, 0.02, "plain", reps=1)
    assert best is None and rows and not any(r["ok"] for r in rows)
