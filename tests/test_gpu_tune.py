"""The autotuner on the GPU: every launch shape of a sweep is timed and checked against
an FP64-reduced run at the built-in shape, the fastest admitted shape is what the table
then serves, and a shape whose result misses the gate is never admitted."""
import numpy as np
import pytest
import torch

from paper_astro_ph_0703100_amd import _lib, api, ics, tune

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(autouse=True)
def committed_table():
    yield
    _lib.nbody_tune_reset()
    _lib.nbody_tune_load(_lib.TUNING_PATH)


def sweep_size(n):
    return sum(1 for _ in tune.IPLS for jt in tune.JTILES for s in tune.SEGS
               if s <= (n + jt - 1) // jt)


def check_sweep(best, rows, n):
    assert len(rows) == sweep_size(n)
    assert all(r["ok"] for r in rows), [r for r in rows if not r["ok"]][:3]
    assert best["ms"] == min(r["ms"] for r in rows)


def test_force_sweep_admits_every_shape_and_the_table_serves_the_best():
    n, eps = 3001, 0.02
    best, rows = tune.tune_force(n, 7, eps, "comp", reps=1)
    check_sweep(best, rows, n)
    _lib.nbody_tune_set(_lib.KERNELS["force"], _lib.PRECISIONS["comp"], n, best["ipl"],
                        best["jtile"], best["nseg"])
    assert _lib.nbody_tune_get(_lib.KERNELS["force"], _lib.PRECISIONS["comp"], n)[:2] == \
        (best["ipl"], best["jtile"])
    pos, _, mass = ics.plummer(n, seed=7)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    a_table, p_table = api.force(p, m, eps)
    a_shape, p_shape = api.force(p, m, eps, ipl=best["ipl"], jtile=best["jtile"],
                                 nseg=best["nseg"])
    torch.cuda.synchronize()
    assert torch.equal(a_table, a_shape) and torch.equal(p_table, p_shape)


def test_jerk_and_vjp_sweeps():
    n = 1500
    best, rows = tune.tune_jerk(n, 8, 0.03, "comp", reps=1)
    check_sweep(best, rows, n)
    best, rows = tune.tune_vjp(n, 9, 0.03, "comp", reps=1)
    check_sweep(best, rows, n)


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
