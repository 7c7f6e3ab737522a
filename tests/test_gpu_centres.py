"""Reference centres for FP64 positions: Morton ordering, per-i-tile centres, and the
precision-stress workload (2^20 particles, a 1e-3-scale core holding 10 % of the mass,
the whole system offset to (1000, 0, 0), eps = 1e-4)."""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _morton_cpu(pos):
    """Z-order by the same quantisation, written independently with numpy."""
    n = len(pos)
    ib = int(np.ceil(np.log2(n))) if n > 1 else 0
    qb = (64 - ib) // 3
    lo, hi = pos.min(0), pos.max(0)
    top = float((1 << qb) - 1)
    q = np.clip((pos - lo) / (hi - lo) * top, 0, top).astype(np.uint64)
    key = np.zeros(n, dtype=np.uint64)
    for b in range(qb):
        for c in range(3):
            key |= ((q[:, c] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 2 - c)
    return np.argsort(key, kind="stable")


def test_morton_order_is_a_spatially_compact_permutation():
    n = 100003
    pos, _, _ = ics.plummer(n, seed=90, velocities=False)
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    perm = api.morton_order(x).cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(n))
    np.testing.assert_array_equal(perm, api.morton_order(x).cpu().numpy())
    np.testing.assert_array_equal(perm, _morton_cpu(pos))
    # Tiles of 256 consecutive particles: median RMS distance to the tile mean.
    def spread(p):
        t = p[: (n // 256) * 256].reshape(-1, 256, 3)
        return float(np.median(np.sqrt(((t - t.mean(1, keepdims=True)) ** 2).sum(-1).mean(1))))
    assert spread(pos[perm]) < 0.25 * spread(pos)
    one = torch.tensor([[1.0], [2.0], [3.0]], dtype=torch.float64, device=DEV)
    assert api.morton_order(one).cpu().tolist() == [0]


@pytest.fixture(scope="module")
def stress():
    w = ics.WORKLOADS["stress_1m"]
    pos, mass, core = ics.stress_system(w.n, seed=w.seed)
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    perm = api.morton_order(x).cpu().numpy().astype(np.int64)
    pos_s, mass_s, core_s = pos[perm], mass[perm], core[perm]
    m32 = mass_s.astype(np.float32)
    idx = ics.stratified_indices(core_s, 2048, seed=w.seed + 1000)
    eps = float(np.float32(w.eps))
    ra, rp = oracle.force_sampled(pos_s, m32.astype(np.float64), eps, idx)
    return {"x": torch.from_numpy(np.ascontiguousarray(pos_s.T)).to(DEV),
            "m": torch.from_numpy(m32).to(DEV), "idx": idx, "core": core_s[idx], "eps": eps,
            "ra": ra, "rp": rp}


@pytest.mark.parametrize("precision", ["comp", "fp64red", "plain"])
def test_stress_1m_centre_modes(stress, precision):
    s = stress
    errs = {}
    for centre in ("tile", "system", "none"):
        acc, pot = api.force_f64(s["x"], s["m"], s["eps"], precision=precision, centre=centre)
        torch.cuda.synchronize()
        a = acc.cpu().numpy().T[s["idx"]]
        e_all = rel_errors(a, s["ra"])
        e_core = rel_errors(a[s["core"]], s["ra"][s["core"]])
        e_halo = rel_errors(a[~s["core"]], s["ra"][~s["core"]])
        ep = rel_errors(pot.cpu().numpy()[s["idx"]], s["rp"])
        errs[centre] = (e_all, e_core, e_halo, ep)
        print(precision, centre, "all %.3e core %.3e halo %.3e (E_max %.3e) pot %.3e" % (
            e_all["rel_rms"], e_core["rel_rms"], e_halo["rel_rms"], e_all["e_max"], ep["rel_rms"]))
    if precision != "plain":
        assert errs["tile"][0]["rel_rms"] <= 1e-6
        assert errs["tile"][3]["rel_rms"] <= 1e-6
    assert errs["tile"][1]["rel_rms"] < errs["system"][1]["rel_rms"]
    assert errs["system"][0]["rel_rms"] < 1e-4
    assert errs["none"][1]["rel_rms"] > 1e-2  # FP32 coordinates near 1000 cannot resolve the core


@pytest.mark.parametrize("precision", ["comp", "fp64red"])
def test_stress_1m_arithmetic_error_apart_from_representation(stress, precision):
    """The same evaluations against the oracle run on the FP32 inputs the kernel sees
    (fp32(x - c), c the FP64 mean of all positions, for the system centre; fp32(x)
    without one): what is left is the kernel's own arithmetic, which stays at the
    force tolerance even where the representation error of the inputs (about 1e-6 with
    the system centre, 1e-2 without) does not."""
    s = stress
    x = s["x"].cpu().numpy().T
    m64 = s["m"].cpu().numpy().astype(np.float64)
    for centre, c in (("system", x.mean(axis=0)), ("none", np.zeros(3))):
        x32 = (x - c).astype(np.float32).astype(np.float64)
        ra, rp = oracle.force_sampled(x32, m64, s["eps"], s["idx"])
        acc, pot = api.force_f64(s["x"], s["m"], s["eps"], precision=precision, centre=centre)
        torch.cuda.synchronize()
        ea = rel_errors(acc.cpu().numpy().T[s["idx"]], ra)
        ep = rel_errors(pot.cpu().numpy()[s["idx"]] , rp)
        e_rep = rel_errors(ra, s["ra"])
        print(precision, centre, "arithmetic %.3e (pot %.3e), representation %.3e"
              % (ea["rel_rms"], ep["rel_rms"], e_rep["rel_rms"]))
        assert ea["rel_rms"] <= 1e-6 and ep["rel_rms"] <= 1e-6


def test_leapfrog_with_tile_centres_matches_oracle():
    n, steps, dt = 3000, 8, 1.0 / 256
    pos, vel, mass = ics.plummer(n, seed=91)
    pos = pos + np.array([300.0, -50.0, 20.0])
    xt = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    perm = api.morton_order(xt).cpu().numpy().astype(np.int64)
    pos, vel, mass = pos[perm], vel[perm], mass[perm]
    m32 = mass.astype(np.float32)
    eps = float(np.float32(0.01))
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(vel.T)).to(DEV)
    m = torch.from_numpy(m32).to(DEV)
    acc, _, _ = api.leapfrog(x, v, m, eps, dt, steps, centre="tile")
    torch.cuda.synchronize()
    xo, vo, ao, _ = oracle.rollout(pos, vel, m32.astype(np.float64), eps, dt, steps)
    assert np.abs(x.cpu().numpy().T - xo).max() < 1e-9
    assert np.abs(v.cpu().numpy().T - vo).max() < 1e-7
    assert rel_errors(acc.cpu().numpy().T, ao)["rel_rms"] < 1e-6
