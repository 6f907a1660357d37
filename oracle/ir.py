"""Iterative-refinement reference -- TEST INFRASTRUCTURE ONLY.

Classical mixed-precision refinement written out plainly: the matrix is
rounded to a lower precision and factored (by the binary64 oracle, on the
rounded matrix), x0 is solved from those factors, then r = b - A x is formed
in binary64 with the original A, the correction solves with the same factors,
and x += d in binary64, until the benchmark's scaled residual is below 16.
The paper itself does not refine (section "High Performance Linpack": no
iterative method is used when running in lower precision); the stopping rules
are this project's reading: stop below 16; give up when the residual is not
finite, grows two steps in a row, or after max_iter corrections.

Used to check the GPU refinement driver's decisions and to calibrate how many
steps a precision needs on the synthetic inputs.
"""
from __future__ import annotations

import math

import numpy as np

from . import getrf, getrs, residual


def round_bf16(a: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 -> binary32, round to nearest even (NaN kept)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out)


def round_to(a: np.ndarray, prec: str) -> np.ndarray:
    a32 = np.asarray(a, dtype=np.float64).astype(np.float32)
    if prec == "fp32":
        return a32
    if prec == "bf16":
        return round_bf16(a32)
    if prec == "fp16":
        return a32.astype(np.float16).astype(np.float32)
    raise ValueError(prec)


def decide(history, corrections: int, max_iter: int) -> int:
    """0: refine again, 1: converged, 2: give up."""
    s = history[-1]
    if not math.isfinite(s):
        return 2
    if s < 16.0:
        return 1
    if len(history) >= 3 and history[-1] > history[-2] > history[-3]:
        return 2
    if corrections >= max_iter:
        return 2
    return 0


def refine(a, b, prec: str = "bf16", max_iter: int = 30):
    """Returns (x, history, converged, corrections) of refinement with factors of
    A rounded to `prec` (whole-matrix rounding: a proxy for the GPU's per-update
    rounding, which is stated where it is used)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(a.shape[0], -1)
    lu, piv, info = getrf(round_to(a, prec).astype(np.float64))
    if info != 0:
        return None, [], False, 0
    x = getrs(lu, piv, b)
    hist = [float(residual(a, x, b)[:, 0].max())]
    k = 0
    while True:
        d = decide(hist, k, max_iter)
        if d == 1:
            return x, hist, True, k
        if d == 2:
            return x, hist, False, k
        r = b - a @ x
        x = x + getrs(lu, piv, r)
        k += 1
        hist.append(float(residual(a, x, b)[:, 0].max()))


# ------------------------------------------------------------------ GMRES-IR
# Refinement whose correction equation A d = r is solved by GMRES on the
# left-preconditioned system (U^-1 L^-1 P A) d = U^-1 L^-1 P r, all in binary64,
# with the low-precision factors only as the preconditioner (E. Carson and
# N. J. Higham, "A new analysis of iterative refinement and its application to
# accurate solution of ill-conditioned sparse linear systems", SIAM J. Sci.
# Comput. 39, 2017; "Accelerating the solution of linear systems by iterative
# refinement in three precisions", SIAM J. Sci. Comput. 40, 2018).  Classical
# refinement needs kappa(A) u_f < 1 for the factorization's unit roundoff u_f;
# GMRES only needs the preconditioned matrix to be reasonably conditioned, so
# refinement keeps converging for much larger kappa(A) u_f.  The paper itself
# does not refine (section "High Performance Linpack"); this is the stronger
# refinement for unshifted inputs in low precision.

def gmres(apply_a, apply_m, r, restart: int, tol: float, max_it: int):
    """GMRES on M^-1 A d = M^-1 r from d = 0, restarted every `restart` steps:
    Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
    matrix, stop when the preconditioned residual norm falls below tol times
    its initial value or after max_it steps.  Returns (d, steps, rel_res)."""
    n = r.shape[0]
    d = np.zeros(n)
    z0 = apply_m(r)
    beta0 = float(np.linalg.norm(z0))
    if beta0 == 0.0:
        return d, 0, 0.0
    steps = 0
    rel = 1.0
    z = z0
    while steps < max_it:
        beta = float(np.linalg.norm(z))
        m = min(restart, max_it - steps)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = z / beta
        k = 0
        for j in range(m):
            w = apply_m(apply_a(V[j]))
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            hnext = H[j + 1, j]
            if hnext != 0.0:
                V[j + 1] = w / hnext
            for i in range(j):  # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            steps += 1
            rel = abs(g[j + 1]) / beta0
            if rel <= tol or hnext == 0.0:  # converged, or the Krylov space is exhausted
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution with the rotated H
            y[i] = (g[i] - float(np.dot(H[i, i + 1:k], y[i + 1:k]))) / H[i, i]
        d = d + V[:k].T @ y
        if rel <= tol:
            break
        z = apply_m(r - apply_a(d))
    return d, steps, rel


def gmres_ir(a, b, prec: str = "bf16", max_iter: int = 30, restart: int = 50,
             tol: float = 1e-8, max_inner: int = 200):
    """GMRES-based refinement with factors of A rounded to `prec` (the same
    whole-matrix rounding proxy as refine()).  b is one right-hand side.
    Returns (x, history, converged, corrections, inner_steps)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    lu, piv, info = getrf(round_to(a, prec).astype(np.float64))
    if info != 0:
        return None, [], False, 0, 0
    apply_m = lambda v: getrs(lu, piv, v)  # noqa: E731
    apply_a = lambda v: a @ v  # noqa: E731
    x = apply_m(b)
    hist = [float(residual(a, x, b)[0, 0])]
    k = 0
    inner = 0
    while True:
        dcs = decide(hist, k, max_iter)
        if dcs == 1:
            return x, hist, True, k, inner
        if dcs == 2:
            return x, hist, False, k, inner
        r = b - a @ x
        d, steps, _ = gmres(apply_a, apply_m, r, restart, tol, max_inner)
        inner += steps
        x = x + d
        k += 1
        hist.append(float(residual(a, x, b)[0, 0]))
