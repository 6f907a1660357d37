"""CPU oracle for the dense LU solve path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it.

It wraps ``oracle.c`` (plain C, binary64, unblocked Gaussian elimination with
partial pivoting, triangular solves and the benchmark's scaled residual; see
that file's header for the exact conventions) through ctypes on numpy arrays,
and ``brute.py`` (exact rational elimination for tiny matrices).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
EPS = 2.0 ** -53

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (contraction off, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_getrf.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, ip]
        lib.orc_getrf.restype = ctypes.c_int
        lib.orc_getrf_nopiv.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip]
        lib.orc_getrf_nopiv.restype = ctypes.c_int
        lib.orc_getrs.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp, ctypes.c_int,
                                  ctypes.c_int]
        lib.orc_getrs.restype = ctypes.c_int
        lib.orc_getrs_trans.argtypes = lib.orc_getrs.argtypes
        lib.orc_getrs_trans.restype = ctypes.c_int
        for name in ("orc_residual", "orc_residual_ld"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                          ctypes.c_int, ctypes.c_int, dp]
            f.restype = None
        lib.orc_row_residuals.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp,
                                          ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp,
                                          dp]
        lib.orc_row_residuals.restype = None
        fp = ctypes.POINTER(ctypes.c_float)
        lib.orc_ptrans.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                   ctypes.c_int]
        lib.orc_ptrans.restype = None
        lib.orc_ptrans_f32.argtypes = [ctypes.c_int, fp, ctypes.c_int, fp, ctypes.c_int, fp,
                                       ctypes.c_int]
        lib.orc_ptrans_f32.restype = None
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _as_f64(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if not a.flags.c_contiguous:
        a = np.ascontiguousarray(a)
    return a


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def getrf(a, overwrite: bool = False):
    """Partial-pivoting LU of an m x n matrix. Returns (LU, ipiv, info)."""
    lib = _load()
    lu = _as_f64(a) if overwrite else np.array(a, dtype=np.float64, order="C", copy=True)
    if lu.ndim != 2:
        raise ValueError("getrf expects a 2-D array")
    m, n = lu.shape
    ipiv = np.zeros(min(m, n), dtype=np.int32)
    info = np.zeros(1, dtype=np.int32)
    rc = lib.orc_getrf(m, n, _dp(lu), max(n, 1), _ip(ipiv), _ip(info))
    if rc != 0:
        raise ValueError(f"orc_getrf rejected argument {-rc}")
    return lu, ipiv, int(info[0])


def getrf_nopiv(a):
    """The paper's elimination without interchanges. Returns (LU, info)."""
    lib = _load()
    lu = np.array(a, dtype=np.float64, order="C", copy=True)
    m, n = lu.shape
    info = np.zeros(1, dtype=np.int32)
    rc = lib.orc_getrf_nopiv(m, n, _dp(lu), max(n, 1), _ip(info))
    if rc != 0:
        raise ValueError(f"orc_getrf_nopiv rejected argument {-rc}")
    return lu, int(info[0])


def getrs(lu, ipiv, b, trans: bool = False):
    """Solve with factors from getrf. b is n or n x nrhs; returns x (same shape).
    trans=True solves A^T x = b with the same factors."""
    lib = _load()
    lu = _as_f64(lu)
    n = lu.shape[0]
    b = np.array(b, dtype=np.float64, copy=True)
    vec = b.ndim == 1
    bb = np.ascontiguousarray(b.reshape(n, -1))
    nrhs = bb.shape[1]
    piv = None if ipiv is None else np.ascontiguousarray(np.asarray(ipiv, dtype=np.int32))
    f = lib.orc_getrs_trans if trans else lib.orc_getrs
    rc = f(n, _dp(lu), max(lu.shape[1], 1),
                       _ip(piv) if piv is not None else None, _dp(bb), max(nrhs, 1), nrhs)
    if rc < 0:
        raise ValueError(f"orc_getrs rejected argument {-rc}")
    if rc == 1:
        raise ZeroDivisionError("singular U: exact zero on the diagonal")
    return bb.reshape(-1) if vec else bb


def solve(a, b):
    lu, ipiv, info = getrf(a)
    if info != 0:
        raise ZeroDivisionError(f"singular matrix, info={info}")
    return getrs(lu, ipiv, b)


def residual(a, x, b, long_double: bool = False) -> np.ndarray:
    """Per-rhs rows of {s, ||r||, ||A||, ||x||, ||b||} (nrhs x 5)."""
    lib = _load()
    a = _as_f64(a)
    n = a.shape[0]
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n, -1))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(n, -1))
    nrhs = x.shape[1]
    out = np.zeros((nrhs, 5), dtype=np.float64)
    f = lib.orc_residual_ld if long_double else lib.orc_residual
    f(n, _dp(a), max(a.shape[1], 1), _dp(x), max(nrhs, 1), _dp(b), max(nrhs, 1), nrhs,
      _dp(out))
    return out


def row_residuals(a_rows, x, b_rows):
    """r_i = sum_j a_ij x_j - b_i and sum_j |a_ij x_j| for the given rows."""
    lib = _load()
    a_rows = _as_f64(a_rows)
    cnt, n = a_rows.shape
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n, -1))
    nrhs = x.shape[1]
    b_rows = np.ascontiguousarray(np.asarray(b_rows, dtype=np.float64).reshape(cnt, nrhs))
    r = np.zeros((cnt, nrhs))
    ad = np.zeros((cnt, nrhs))
    lib.orc_row_residuals(n, cnt, _dp(a_rows), n, _dp(x), nrhs, _dp(b_rows), nrhs, nrhs,
                          _dp(r), _dp(ad))
    return r, ad


def ptrans(a, b):
    """C = B + A^T (the paper's PTRANS), in the precision of a (float64 or float32)."""
    lib = _load()
    if np.asarray(a).dtype == np.float32:
        a = np.ascontiguousarray(a, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        c = np.empty_like(b)
        fp = ctypes.POINTER(ctypes.c_float)
        n = a.shape[0]
        lib.orc_ptrans_f32(n, a.ctypes.data_as(fp), max(n, 1), b.ctypes.data_as(fp), max(n, 1),
                           c.ctypes.data_as(fp), max(n, 1))
        return c
    a = _as_f64(a)
    b = _as_f64(b)
    c = np.empty_like(b)
    n = a.shape[0]
    lib.orc_ptrans(n, _dp(a), max(n, 1), _dp(b), max(n, 1), _dp(c), max(n, 1))
    return c


def unpack(lu):
    """Split packed factors into (L unit lower, U upper) dense arrays."""
    lu = np.asarray(lu)
    m, n = lu.shape
    k = min(m, n)
    L = np.tril(lu[:, :k], -1) + np.eye(m, k)
    U = np.triu(lu[:k, :])
    return L, U


def perm_from_ipiv(ipiv, m: int) -> np.ndarray:
    """Row order p such that (P A)[i] = A[p[i]] after the sequential swaps."""
    p = np.arange(m)
    for k, r in enumerate(np.asarray(ipiv)):
        if r != k:
            p[[k, r]] = p[[r, k]]
    return p


def flops(n: int, nrhs: int = 1) -> float:
    """Operation count of factor + solve: 2/3 n^3 + 2 n^2 per right-hand side."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n ** 2 * nrhs
