"""Accuracy and throughput figures used to report results.

Per-particle relative error e_i = |a_i - a_ref,i| / |a_ref,i|.  The paper reports
the maximum of e_i over all particles (Sec. 3.4, eq. (3)); the relative RMS is
sqrt(mean e_i^2); the normwise error is ||a - a_ref||_2 / ||a_ref||_2.  For a
scalar per particle (the potential) |.| is the absolute value.

Flop conventions: the paper counts "about 20" floating-point operations per pair
(Sec. 1.1) and quotes its Gflop/s with 38 per pair (Sec. 3.5, eq. (4)).
"""
from __future__ import annotations

import numpy as np

FLOPS_PER_PAIR_PAPER = 38   # eq. (4) convention
FLOPS_PER_PAIR_OPS = 20     # the paper's own operation count


def rel_errors(approx, exact) -> dict:
    """Relative RMS, maximum (eq. (3)) and normwise error of ``approx`` against ``exact``.

    Arrays are (n, 3) vectors or (n,) scalars.  Rows whose reference is exactly
    zero are left out of the per-particle statistics.
    """
    a = np.asarray(approx, dtype=np.float64)
    b = np.asarray(exact, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("shape mismatch %s vs %s" % (a.shape, b.shape))
    if a.ndim == 1:
        a = a[:, None]
        b = b[:, None]
    d = np.linalg.norm(a - b, axis=1)
    r = np.linalg.norm(b, axis=1)
    ok = r > 0
    e = d[ok] / r[ok]
    if e.size == 0:
        return {"rel_rms": 0.0, "e_max": 0.0, "normwise": 0.0, "count": 0}
    nb = float(np.linalg.norm(b))
    return {
        "rel_rms": float(np.sqrt(np.mean(e * e))),
        "e_max": float(e.max()),
        "normwise": float(np.linalg.norm(a - b) / nb) if nb > 0 else 0.0,
        "count": int(e.size),
    }


def gflops(pairs: float, seconds: float, flops_per_pair: int = FLOPS_PER_PAIR_PAPER) -> float:
    """S = n_flo * pairs / t in Gflop/s (eq. (4) with pairs = N^2)."""
    return flops_per_pair * pairs / seconds / 1e9
