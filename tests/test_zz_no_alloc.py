"""nbody_force_noalloc (static device scratch, no allocation) against nbody_force_ex on
the GPU: the same launch shape gives bitwise the same result; the automatic shape (the
grid engine's j-split shortened to fit the static array) agrees with nbody_force_ex and
with the FP64 oracle to the force tolerance.  Two calls in a row, the second smaller, so
the second reads partial sums its own kernels wrote, not the first call's."""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0703100_amd import _lib, api, ics
from paper_astro_ph_0703100_amd.metrics import rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def inputs(n, seed):
    pos, _, mass = ics.plummer(n, seed=seed, velocities=False)
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    return torch.from_numpy(p32).to(DEV), torch.from_numpy(m32).to(DEV), p32, m32


def noalloc(n, p, m, eps, opts):
    acc = torch.full((3, n), np.nan, dtype=torch.float64, device=DEV)
    pot = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    _lib.nbody_force_noalloc(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), pot.data_ptr(),
                             opts, api.stream_ptr())
    return acc, pot


def ex(n, p, m, eps, opts):
    acc = torch.empty((3, n), dtype=torch.float64, device=DEV)
    pot = torch.empty((n,), dtype=torch.float64, device=DEV)
    _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), pot.data_ptr(), opts,
                        api.stream_ptr())
    return acc, pot


@pytest.mark.parametrize("shape", [dict(ipl=1, jtile=256, nseg=40, jlanes=1),
                                   dict(ipl=2, jtile=128, nseg=7, jlanes=1),
                                   dict(ipl=1, jtile=512, jlanes=64),
                                   dict(ipl=4, jtile=64, nseg=8, symmetric=2)])
def test_noalloc_matches_force_ex_bitwise_on_two_calls(shape):
    eps = 0.01
    for n, seed in ((40000, 1), (5003, 2)):  # second call smaller
        p, m, _, _ = inputs(n, seed)
        for prec in ("comp", "plain"):
            o = api.make_opts(precision=prec, **shape)
            a1, p1 = noalloc(n, p, m, eps, o)
            a2, p2 = ex(n, p, m, eps, o)
            torch.cuda.synchronize()
            assert torch.equal(a1, a2) and torch.equal(p1, p2), (shape, n, prec)


def test_noalloc_default_shape_at_the_paper_size_then_smaller():
    """N = 131072 (its tuned j-split needs more than the static array: fewer, longer
    segments are used) and then N = 3001; both against nbody_force_ex and the oracle."""
    w = ics.WORKLOADS["plummer_131072"]
    eps = float(np.float32(w.eps))
    for n, seed in ((w.n, w.seed), (3001, 9)):
        p, m, p32, m32 = inputs(n, seed)
        o = api.make_opts()
        a1, q1 = noalloc(n, p, m, eps, o)
        a2, q2 = ex(n, p, m, eps, o)
        torch.cuda.synchronize()
        a1, q1 = a1.cpu().numpy().T, q1.cpu().numpy()
        a2, q2 = a2.cpu().numpy().T, q2.cpu().numpy()
        assert np.all(np.isfinite(a1)) and np.all(np.isfinite(q1))
        assert rel_errors(a1, a2)["rel_rms"] <= 1e-6 and rel_errors(q1, q2)["rel_rms"] <= 1e-6
        idx = ics.sample_indices(n, min(n, 1024), seed=seed + 1000)
        ra, rp = oracle.force_sampled(p32.T.astype(np.float64), m32.astype(np.float64), eps, idx)
        assert rel_errors(a1[idx], ra)["rel_rms"] <= 1e-6
        assert rel_errors(q1[idx], rp)["rel_rms"] <= 1e-6


def test_noalloc_symmetric_table_entry_falls_back_to_the_grid_engine():
    """A tuned symmetric-engine shape whose j-side sums do not fit the static array
    (N = 131072) is replaced by the grid engine's; an explicit symmetric = 2 is refused."""
    w = ics.WORKLOADS["plummer_131072"]
    eps = float(np.float32(w.eps))
    p, m, _, _ = inputs(w.n, w.seed)
    try:
        _lib.nbody_tune_set(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, w.n, 4, 64, 0, 1, 1)
        a1, q1 = noalloc(w.n, p, m, eps, api.make_opts())
        a2, q2 = ex(w.n, p, m, eps, api.make_opts(symmetric=1))
        torch.cuda.synchronize()
        assert rel_errors(a1.cpu().numpy().T, a2.cpu().numpy().T)["rel_rms"] <= 1e-6
        assert rel_errors(q1.cpu().numpy(), q2.cpu().numpy())["rel_rms"] <= 1e-6
        with pytest.raises(_lib.NBodyError) as e:
            noalloc(w.n, p, m, eps, api.make_opts(symmetric=2))
        assert e.value.status == _lib.NBODY_EINVAL and "static scratch" in str(e.value)
    finally:
        _lib.nbody_tune_reset()
        _lib.nbody_tune_load(_lib.TUNING_PATH)
