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
