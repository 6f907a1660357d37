"""Seeded synthetic inputs for the dense linear solver (host side).

The workload of the LINPACK benchmark (paper, section "High Performance Linpack")
is a dense n x n system A x = b.  The paper builds A so that x is all ones; the
synthetic recipe used here instead draws A and b i.i.d. uniform on [-0.5, 0.5)
from a seed, optionally adding n to every diagonal entry (the diagonally
dominant HPL-AI form the paper adopts, for which pivoting is not needed).

Generator: a counter-based SplitMix64 stream (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).  For a given
(seed, stream) the generator state starts at

    key = mix64(seed) XOR (stream << 60)

and the idx-th 64-bit word is the SplitMix64 output for that state advanced
idx+1 times by the golden gamma:

    word(idx) = mix64(key + (idx + 1) * 0x9E3779B97F4A7C15)      (mod 2**64)
    mix64(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31

and the value is (word >> 11) * 2**-53 - 0.5, exact in binary64.
Stream 0 is the matrix A with idx = i*n + j; stream 1 is the right-hand side
B (n x nrhs) with idx = i*nrhs + c.  The diagonal shift is fl(a_ii + shift)
in round-to-nearest binary64.

This module holds none of the solver's arithmetic.  Both the CPU oracle and
the GPU path take their inputs from here: this file is the host generator
(numpy); ``inputs/gen.hip`` is the same generator as a device kernel, loaded
through :func:`device`.  The two are checked bitwise against each other.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
STREAM_A = 0
STREAM_B = 1
_M64 = (1 << 64) - 1

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libinputs_gen.so")


def mix64_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (reference for the vector form)."""
    z &= _M64
    z ^= z >> 30
    z = (z * MIX1) & _M64
    z ^= z >> 27
    z = (z * MIX2) & _M64
    z ^= z >> 31
    return z


def stream_key(seed: int, stream: int) -> int:
    return mix64_int(seed) ^ ((stream << 60) & _M64)


def _mix64_vec(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(MIX1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(MIX2)
    z = z ^ (z >> np.uint64(31))
    return z


def words(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """64-bit words for counter indices ``idx`` (uint64 array)."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = key + (idx + np.uint64(1)) * np.uint64(GOLDEN)
        return _mix64_vec(state)


def uniform(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Values in [-0.5, 0.5) for counter indices ``idx``."""
    w = words(seed, stream, idx)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5


def matrix_rows(seed: int, n: int, rows, shift: float = 0.0) -> np.ndarray:
    """Rows ``rows`` (iterable of row indices) of the n x n matrix A."""
    rows = np.asarray(list(rows) if not isinstance(rows, np.ndarray) else rows,
                      dtype=np.int64)
    out = np.empty((rows.size, n), dtype=np.float64)
    cols = np.arange(n, dtype=np.uint64)
    for t, i in enumerate(rows):
        out[t] = uniform(seed, STREAM_A, np.uint64(i) * np.uint64(n) + cols)
        if shift != 0.0:
            out[t, i] = out[t, i] + shift
    return out


def matrix(seed: int, n: int, shift: float = 0.0, chunk_rows: int = 1024) -> np.ndarray:
    """The full n x n matrix A (row-major float64)."""
    a = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        idx = (np.arange(r0, r1, dtype=np.uint64)[:, None] * np.uint64(n)
               + np.arange(n, dtype=np.uint64)[None, :])
        a[r0:r1] = uniform(seed, STREAM_A, idx)
    if shift != 0.0:
        d = np.arange(n)
        a[d, d] = a[d, d] + shift
    return a


def rhs(seed: int, n: int, nrhs: int = 1) -> np.ndarray:
    """The n x nrhs right-hand side B (row-major float64)."""
    idx = (np.arange(n, dtype=np.uint64)[:, None] * np.uint64(nrhs)
           + np.arange(nrhs, dtype=np.uint64)[None, :])
    return uniform(seed, STREAM_B, idx)


class _Device:
    """ctypes view of the device generator library (no solver arithmetic)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(
                f"device input generator not built: {path} (run __graft_entry__.build())")
        self.lib = ctypes.CDLL(path)
        f = self.lib.lp_gen_uniform
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int, ctypes.c_int,
                      ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p]

    def fill(self, out_ptr: int, rows: int, cols: int, ld: int, row0: int,
             logical_cols: int, seed: int, stream: int, shift: float,
             is_f32: bool, hip_stream: int) -> None:
        rc = self.lib.lp_gen_uniform(out_ptr, rows, cols, ld, row0, logical_cols,
                                     1 if is_f32 else 0, 0, seed, stream, shift,
                                     hip_stream)
        if rc != 0:
            raise RuntimeError(f"lp_gen_uniform failed with code {rc}")


_DEV = None


def device() -> _Device:
    global _DEV
    if _DEV is None:
        _DEV = _Device()
    return _DEV


def fill_matrix_(t, seed: int, shift: float = 0.0, stream=None, row0: int = 0,
                 logical_cols: int | None = None) -> None:
    """Fill a CUDA tensor (rows x cols, row-major, float64 or float32) with rows
    row0.. of A (stream 0) on the device."""
    import torch
    assert t.is_cuda and t.dim() == 2 and t.stride(1) == 1
    rows, cols = t.shape
    st = (stream or torch.cuda.current_stream()).cuda_stream
    device().fill(t.data_ptr(), rows, cols, t.stride(0), row0,
                  cols if logical_cols is None else logical_cols, seed, STREAM_A,
                  shift, t.dtype == torch.float32, st)


def fill_rhs_(t, seed: int, stream=None) -> None:
    """Fill a CUDA tensor (n x nrhs, row-major) with B (stream 1) on the device."""
    import torch
    assert t.is_cuda and t.dim() == 2 and t.stride(1) == 1
    rows, cols = t.shape
    st = (stream or torch.cuda.current_stream()).cuda_stream
    device().fill(t.data_ptr(), rows, cols, t.stride(0), 0, cols, seed, STREAM_B,
                  0.0, t.dtype == torch.float32, st)
