"""Condition estimate for the oracle's factors -- TEST INFRASTRUCTURE ONLY.

The forward error of a computed solution is bounded by about kappa(A) times
the backward error, so a GPU-versus-oracle difference in x is only meaningful
next to kappa_inf(A) = ||A||_inf ||A^-1||_inf.  Forming A^-1 costs n^3 and n^2
memory, so ||A^-1||_inf is estimated from the oracle's P A = L U with a few
solves: Hager's one-norm estimator with Higham's refinements (W. W. Hager,
"Condition estimates", SIAM J. Sci. Stat. Comput. 5, 1984; N. J. Higham,
"FORTRAN codes for estimating the one-norm of a real or complex matrix, with
applications to condition estimation", ACM TOMS 14, 1988, Algorithm 4.1).

||A^-1||_inf = ||A^-T||_1, so the estimator runs on B = A^-T: a product B v is
the transposed solve A^T y = v, a product B^T v the ordinary solve A y = v.
The estimate never exceeds the true norm (up to rounding) and equals it for
most matrices.
"""
from __future__ import annotations

import numpy as np

from . import getrs


def _sign(v: np.ndarray) -> np.ndarray:
    return np.where(v >= 0.0, 1.0, -1.0)


def norm1_estimate(apply_b, apply_bt, n: int, max_iter: int = 5) -> float:
    """Estimate ||B||_1 from products with B and B^T (Higham's Algorithm 4.1)."""
    if n == 0:
        return 0.0
    x = np.full(n, 1.0 / n)
    y = apply_b(x)
    est = float(np.abs(y).sum())
    if n == 1:
        return est
    xi = _sign(y)
    z = apply_bt(xi)
    j = int(np.argmax(np.abs(z)))
    for _ in range(1, max_iter):
        x = np.zeros(n)
        x[j] = 1.0
        y = apply_b(x)
        est_old = est
        est = float(np.abs(y).sum())
        xi_new = _sign(y)
        if np.array_equal(xi_new, xi) or est <= est_old:
            est = max(est, est_old)
            break
        xi = xi_new
        z = apply_bt(xi)
        j_old = j
        j = int(np.argmax(np.abs(z)))
        if abs(z[j]) == abs(z[j_old]):
            break
    # Higham's extra vector: alternating signs with growing magnitude, which
    # catches matrices on which the iteration above stalls
    i = np.arange(n, dtype=np.float64)
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * (1.0 + i / (n - 1))
    alt_est = 2.0 * float(np.abs(apply_b(alt)).sum()) / (3.0 * n)
    return max(est, alt_est)


def inv_norm_inf_estimate(lu: np.ndarray, ipiv) -> float:
    """Estimate of ||A^-1||_inf from the oracle's factors (getrf output)."""
    n = lu.shape[0]
    return norm1_estimate(lambda v: getrs(lu, ipiv, v, trans=True),
                          lambda v: getrs(lu, ipiv, v), n)


def kappa_inf_estimate(anorm_inf: float, lu: np.ndarray, ipiv) -> float:
    """kappa_inf(A) ~= ||A||_inf * estimate of ||A^-1||_inf."""
    return float(anorm_inf) * inv_norm_inf_estimate(lu, ipiv)
