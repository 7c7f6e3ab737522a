"""Per-particle rounding bounds of the FP32 gravity pair kernels against the FP64 oracle.

Both sides see the same FP32 inputs (the oracle promoted to FP64), so the difference
is the kernel's own rounding.  One pair term of eq. (1), with u = 2^-24:

  d = fl(x_j - x_i)                      relative error <= u
  s^2 = three FMAs with eps^2            <= 3 u, plus 2 u from d   -> 5 u
  r = v_rsq_f32(s^2)                     1 ulp (<= 2 u) + 5u / 2   -> 4.5 u
  m r                                    4.5 u + u                 -> 5.5 u   (potential term)
  r r                                    2 * 4.5 u + u             -> 10 u
  (m r)(r r)                             5.5 u + 10 u + u          -> 16.5 u
  ... * d inside the FMA                 + u (d)                   -> 17.5 u  (acceleration term)

so each acceleration component's term errs by at most C_ACC u |t| and each potential
term by C_POT u |t|.  The FP32 additions of a block of B terms add at most (B - 1) u
sum |t|; the compensated mode keeps each block sum exactly after that (two-sum), the
FP64-reduced mode adds it in FP64, so A = 127 more (128-term blocks).  Plain FP32 sums a
whole segment and then the segments in FP32: A < n + 1024.  Hence, per particle and
component,

  |a_c - a_c,ref| <= (C_ACC + A) u sum_j |m_j d_c| / s^3
  |phi - phi_ref| <= (C_POT + A) u sum_j |m_j| / s,

the magnitude sums coming from oracle.force_abs over the same pairs.
"""
import numpy as np

U = 2.0 ** -24
C_ACC = 18.0
C_POT = 6.0
BLOCK_J = 128


def adds(precision, n):
    """FP32 additions a term can pass through after it is formed."""
    return BLOCK_J - 1 if precision != "plain" else n + 1024


def check_acc(acc, ref, absa, precision, n):
    """Asserts the per-component bound; returns the largest error / (u * absa)."""
    ratio = np.abs(acc - ref) / (U * np.maximum(absa, 1e-300))
    worst = float(ratio.max()) if ratio.size else 0.0
    assert worst <= C_ACC + adds(precision, n), (precision, worst)
    return worst


def check_pot(pot, ref, absp, precision, n):
    """Asserts the per-particle potential bound; returns the largest error / (u * absp)."""
    ratio = np.abs(pot - ref) / (U * np.maximum(absp, 1e-300))
    worst = float(ratio.max()) if ratio.size else 0.0
    assert worst <= C_POT + adds(precision, n), (precision, worst)
    return worst
