"""The oracle's rollout gradient at the full differentiation workload, pinned by FP64
central finite differences (CPU only; about 160 oracle rollouts, 1.4e12 pair terms).

Workload: N = 16384 Plummer sphere (a = 1, M = 1, equal masses rounded to FP32, seed 5,
distribution-function velocities), eps = 0.01, 32 KDK steps of dt = 1/256, loss
L = (1/N) sum_i |x_i(T) - y_i|^2 with y = x0 + 0.01 xi, xi ~ N(0, I) (seed 5001).
The GPU gradient is compared with ``oracle.rollout_loss_grad`` on this workload by the
GPU tests; this file checks that oracle gradient itself against central differences
of ``oracle.rollout`` (h = 1e-6 on 64 seeded position coordinates; h = 1e-6 m_k on 16
seeded masses), so the whole chain GPU -> oracle -> FD holds at the stated size.

Tolerance.  The central difference's truncation error (h^2 L'''/6) is far below
1e-12 here; what limits it is rounding: two rollouts whose inputs differ by h round
differently everywhere, so each difference carries the loss's rounding noise dL.
That noise is measured: the loss is recomputed from inputs nudged by a few ulps (a
change whose exact effect on L is ~1e-21, far below dL), and the spread gives dL.
A coordinate passes if |fd - g| <= 1e-6 max|g| + 4 dL / h, with 1e-6 the oracle-vs-FD
bound and dL / h the FD's rounding noise at step h.

Runs only with NBODY_SLOW=1 (about 25 minutes on 8 host threads).
"""
import os
import time

import numpy as np
import pytest

import oracle
from paper_astro_ph_0703100_amd import ics

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("NBODY_SLOW") != "1",
                                 reason="full-size finite differences take ~25 min; set NBODY_SLOW=1")]


def _workload():
    w = ics.WORKLOADS["adjoint_16384"]
    x0, v0, mass = ics.plummer(w.n, seed=w.seed)
    m = mass.astype(np.float32).astype(np.float64)
    y = ics.perturbed_target(x0, seed=5001)
    return w, x0, v0, m, float(np.float32(w.eps)), y


def test_rollout_gradient_adjoint_16384_against_central_differences():
    w, x0, v0, m, eps, y = _workload()
    n = w.n
    t0 = time.perf_counter()
    loss, gx, gv, gm = oracle.rollout_loss_grad(x0, v0, m, eps, w.dt, w.steps, y)
    print("reverse mode: L = %.17g (%.1f s)" % (loss, time.perf_counter() - t0), flush=True)

    def L(xx, mm):
        xT, _, _, _ = oracle.rollout(xx, v0, mm, eps, w.dt, w.steps)
        return float(np.sum((xT - y) ** 2) / n)

    assert abs(L(x0, m) - loss) <= 1e-14 * loss

    # Rounding noise of the loss: inputs nudged by a few ulps in one coordinate each.
    rng_noise = np.random.default_rng(5003)
    spread = []
    for _ in range(3):
        k, c = int(rng_noise.integers(n)), int(rng_noise.integers(3))
        xn = x0.copy()
        xn[k, c] = np.nextafter(np.nextafter(xn[k, c], np.inf), np.inf)
        spread.append(abs(L(xn, m) - loss))
    dL = max(max(spread), 1e-300)
    print("loss rounding noise dL = %.3e (samples %s)" % (dL, spread), flush=True)

    rng = np.random.default_rng(5002)
    h = 1e-6
    coords = [(int(rng.integers(n)), int(rng.integers(3))) for _ in range(64)]
    scale_x = max(abs(gx[k, c]) for k, c in coords)
    worst_x = 0.0
    for q, (k, c) in enumerate(coords):
        xp, xm = x0.copy(), x0.copy()
        xp[k, c] += h
        xm[k, c] -= h
        fd = (L(xp, m) - L(xm, m)) / (2 * h)
        dev = abs(fd - gx[k, c])
        bound = 1e-6 * scale_x + 4 * dL / h
        worst_x = max(worst_x, dev / bound)
        print("x[%5d,%d] fd %+.12e  grad %+.12e  |diff| %.2e  bound %.2e"
              % (k, c, fd, gx[k, c], dev, bound), flush=True)
        assert dev <= bound, (q, k, c, fd, gx[k, c])

    ks = [int(k) for k in rng.choice(n, size=16, replace=False)]
    scale_m = max(abs(gm[k]) for k in ks)
    worst_m = 0.0
    for k in ks:
        hm = 1e-6 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += hm
        mm[k] -= hm
        fd = (L(x0, mp) - L(x0, mm)) / (2 * hm)
        dev = abs(fd - gm[k])
        bound = 1e-6 * scale_m + 4 * dL / hm
        worst_m = max(worst_m, dev / bound)
        print("m[%5d]   fd %+.12e  grad %+.12e  |diff| %.2e  bound %.2e"
              % (k, fd, gm[k], dev, bound), flush=True)
        assert dev <= bound, (k, fd, gm[k])
    print("worst |diff| / bound: positions %.3f, masses %.3f" % (worst_x, worst_m))


def test_rollout_mass_gradient_adjoint_16384_wider_step():
    # The same 16 masses (the same seeded draw) with h = 1e-3 m_k: the difference quotient's
    # rounding noise dL / h is 1000 times smaller than at h = 1e-6 m_k, where it limits
    # the check to about 1e-4 of max |dL/dm|; the truncation error h^2 L''' / 6 stays far
    # below it, L being smooth in each mass (its gravity enters linearly in the forces).
    w, x0, v0, m, eps, y = _workload()
    n = w.n
    loss, _, _, gm = oracle.rollout_loss_grad(x0, v0, m, eps, w.dt, w.steps, y)

    def L(mm):
        xT, _, _, _ = oracle.rollout(x0, v0, mm, eps, w.dt, w.steps)
        return float(np.sum((xT - y) ** 2) / n)

    rng_noise = np.random.default_rng(5003)
    spread = []
    for _ in range(3):
        k, c = int(rng_noise.integers(n)), int(rng_noise.integers(3))
        xn = x0.copy()
        xn[k, c] = np.nextafter(np.nextafter(xn[k, c], np.inf), np.inf)
        xT, _, _, _ = oracle.rollout(xn, v0, m, eps, w.dt, w.steps)
        spread.append(abs(float(np.sum((xT - y) ** 2) / n) - loss))
    dL = max(max(spread), 1e-300)

    rng = np.random.default_rng(5002)
    _ = [(int(rng.integers(n)), int(rng.integers(3))) for _ in range(64)]  # the coordinates' draws
    ks = [int(k) for k in rng.choice(n, size=16, replace=False)]
    scale_m = max(abs(gm[k]) for k in ks)
    worst = 0.0
    for k in ks:
        hm = 1e-3 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += hm
        mm[k] -= hm
        fd = (L(mp) - L(mm)) / (2 * hm)
        dev = abs(fd - gm[k])
        bound = 1e-6 * scale_m + 4 * dL / hm
        worst = max(worst, dev / scale_m)
        print("m[%5d]   fd %+.12e  grad %+.12e  |diff| %.2e  bound %.2e"
              % (k, fd, gm[k], dev, bound), flush=True)
        assert dev <= bound, (k, fd, gm[k])
    print("worst |diff| / max|grad|: %.3e" % worst)
