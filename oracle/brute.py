"""Exact rational elimination for tiny matrices -- TEST INFRASTRUCTURE ONLY.

Gaussian elimination with partial pivoting over ``fractions.Fraction``: every
|a_ik| comparison, division and update is exact, so the pivot sequence, L and
U are the mathematically defined ones (paper, section "High Performance
Linpack": A = L U, then L y = b and U x = y; pivoting as in the textbook
method, smallest row index among equal magnitudes).  Used to pin the binary64
oracle on inputs small enough for exact arithmetic.
"""
from __future__ import annotations

from fractions import Fraction


def to_fractions(a):
    return [[Fraction(v) for v in row] for row in a]


def getrf_exact(a):
    """Returns (LU as list of lists of Fraction, ipiv list, info)."""
    lu = to_fractions(a)
    m = len(lu)
    n = len(lu[0]) if m else 0
    ipiv = []
    info = 0
    for k in range(min(m, n)):
        p = k
        for i in range(k + 1, m):
            if abs(lu[i][k]) > abs(lu[p][k]):
                p = i
        ipiv.append(p)
        if lu[p][k] == 0:
            if info == 0:
                info = k + 1
            continue
        lu[k], lu[p] = lu[p], lu[k]
        for i in range(k + 1, m):
            lu[i][k] = lu[i][k] / lu[k][k]
            for j in range(k + 1, n):
                lu[i][j] = lu[i][j] - lu[i][k] * lu[k][j]
    return lu, ipiv, info


def inverse_exact(a):
    """Gauss-Jordan inverse with exact arithmetic (raises on singular input)."""
    n = len(a)
    m = [to_fractions([row])[0] + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(a)]
    for k in range(n):
        p = next((i for i in range(k, n) if m[i][k] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular")
        m[k], m[p] = m[p], m[k]
        piv = m[k][k]
        m[k] = [v / piv for v in m[k]]
        for i in range(n):
            if i != k and m[i][k] != 0:
                f = m[i][k]
                m[i] = [vi - f * vk for vi, vk in zip(m[i], m[k])]
    return [row[n:] for row in m]


def solve_exact(a, b):
    """x = A^-1 b exactly (b a list of numbers)."""
    inv = inverse_exact(a)
    bf = [Fraction(v) for v in b]
    return [sum((inv[i][j] * bf[j] for j in range(len(bf))), Fraction(0))
            for i in range(len(bf))]


def det_exact(a):
    """Determinant by exact elimination."""
    lu, ipiv, info = getrf_exact(a)
    if info:
        return Fraction(0)
    d = Fraction(1)
    sign = 1
    for k, p in enumerate(ipiv):
        if p != k:
            sign = -sign
        d *= lu[k][k]
    return sign * d
