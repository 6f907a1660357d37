"""MI355X (gfx950) dense LU solver: Python binding of liblp.so.

Argument marshalling only: every step of the factorization, the solves and the
residual check runs in the HIP kernels of ``liblp.so`` (``include/lp.h``).
PyTorch supplies device memory and the current HIP stream.  Importing this
package loads the library and raises if it has not been built
(``python -m paper_2202_13995_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblp.so")

FP64, FP32, BF16, FP16 = 0, 1, 2, 3
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16}
LP_OK = 0
LP_ENOSPC = -900
LP_ENOTSUP = -901
INFO_BARRIER_TIMEOUT = -77


class LPError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {code} ({strerror(code)})")
        self.code = code


class IRReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("fell_back", ctypes.c_int), ("info", ctypes.c_int),
                ("fallback_info", ctypes.c_int), ("history_len", ctypes.c_int),
                ("scaled_residual", ctypes.c_double), ("history", ctypes.c_double * 64),
                ("t_convert_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
                ("t_solve0_ms", ctypes.c_double), ("t_refine_ms", ctypes.c_double),
                ("t_fallback_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("gmres_corrections", ctypes.c_int), ("gmres_steps", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history"}
        d["history"] = [self.history[i] for i in range(self.history_len)]
        return d


class IROpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("gmres", ctypes.c_int),
                ("gmres_restart", ctypes.c_int), ("gmres_max_inner", ctypes.c_int),
                ("gmres_tol", ctypes.c_double), ("no_lookahead", ctypes.c_int)]


class FactorOpts(ctypes.Structure):
    _fields_ = [("lookahead", ctypes.c_int), ("panel_cus", ctypes.c_int),
                ("panel_rows", ctypes.c_int), ("no_pivoting", ctypes.c_int),
                ("panel_split_rows", ctypes.c_int)]


class FactorProfile(ctypes.Structure):
    _fields_ = [("gemm_launches", ctypes.c_int), ("panel_launches", ctypes.c_int),
                ("gemm_ms", ctypes.c_double), ("gemm_flops", ctypes.c_double),
                ("gemm_bytes", ctypes.c_double), ("panel_ms", ctypes.c_double),
                ("swap_ms", ctypes.c_double), ("swap_bytes", ctypes.c_double),
                ("trsm_ms", ctypes.c_double), ("trsm_flops", ctypes.c_double),
                ("swap_left_ms", ctypes.c_double), ("swap_left_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    _fields_ = [("memory_bytes", ctypes.c_size_t), ("small_n_max", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("batch_slots", ctypes.c_int),
                ("batch_workgroups", ctypes.c_int), ("large_slots", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("lda", ctypes.c_int), ("ldb", ctypes.c_int), ("ldx", ctypes.c_int),
                ("n", ctypes.c_int), ("nrhs", ctypes.c_int), ("prec", ctypes.c_int),
                ("nb", ctypes.c_int), ("max_iter", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int), ("info", ctypes.c_int),
                ("iterations", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("batched", ctypes.c_int), ("scaled_residual", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("device_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_D = ctypes.c_double

# name -> (restype, argtypes); the order follows include/lp.h
SIGNATURES = {
    "lp_strerror": (ctypes.c_char_p, [_I]),
    "lp_version": (_I, []),
    "lu_workspace_bytes": (_SZ, [_I, _I, _I]),
    "lu_factor": (_I, [_I, _I, _I, _VP, _I, _VP, _VP, _VP, _SZ, _VP]),
    "lu_factor_ex": (_I, [_I, _I, _I, _VP, _I, _VP, _VP, _VP, _SZ, ctypes.POINTER(FactorOpts),
                          ctypes.POINTER(FactorProfile), _VP]),
    "lu_factor_noalloc_max_bytes": (_SZ, []),
    "lu_factor_noalloc": (_I, [_I, _I, _I, _VP, _I, _VP, _VP, _VP]),
    "lu_factor_nopiv": (_I, [_I, _I, _I, _VP, _I, _VP, _VP, _VP, _SZ, _VP]),
    "lu_solve": (_I, [_I, _I, _VP, _I, _VP, _VP, _VP, _I, _I, _VP, _VP]),
    "lu_solve_workspace_bytes": (_SZ, [_I, _I, _I]),
    "lu_solve_ex": (_I, [_I, _I, _VP, _I, _VP, _VP, _VP, _I, _I, _VP, _VP, _SZ, _VP]),
    "residual_check": (_I, [_I, _VP, _I, _VP, _I, _VP, _I, _I, _VP, _VP]),
    "lu_solve_ir_workspace_bytes": (_SZ, [_I, _I, _I, _I]),
    "lu_solve_ir": (_I, [_I, _I, _I, _VP, _I, _VP, _I, _VP, _I, _I, _I, _VP, _SZ,
                         ctypes.POINTER(IRReport), _VP]),
    "lu_solve_ir_ex": (_I, [_I, _I, _I, _VP, _I, _VP, _I, _VP, _I, _I, ctypes.POINTER(IROpts),
                            _VP, _SZ, ctypes.POINTER(IRReport), _VP]),
    "lp_server_create": (_I, [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]),
    "lp_server_destroy": (_I, [_VP]),
    "lp_server_submit": (_I, [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64),
                              _VP]),
    "lp_server_poll": (_I, [_VP, ctypes.POINTER(Result), _I, ctypes.POINTER(ctypes.c_int)]),
    "lp_server_pending": (_I, [_VP, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_size_t)]),
    "lp_request_footprint": (_SZ, [ctypes.POINTER(ServerCfg), ctypes.POINTER(Request)]),
    "lp_ir_decide": (_I, [ctypes.POINTER(ctypes.c_double), _I, _I, _I]),
    "lp_panel_factor": (_I, [_I, _I, _I, _VP, _I, _VP, _VP, _VP, _SZ, _I, _VP]),
    "lp_laswp_workspace_bytes": (_SZ, [_I]),
    "lp_laswp": (_I, [_I, _VP, _I, _I, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "lp_trsm_workspace_bytes": (_SZ, [_I]),
    "lp_trsm_lower_unit": (_I, [_I, _I, _I, _VP, _I, _VP, _I, _VP, _SZ, _VP]),
    "lp_trsm_right_workspace_bytes": (_SZ, [_I]),
    "lp_trsm_right_upper": (_I, [_I, _I, _I, _VP, _I, _VP, _I, _VP, _SZ, _VP]),
    "lp_gemm_update": (_I, [_I, _I, _I, _I, _VP, _I, _VP, _I, _VP, _I, _VP]),
    "lp_gemm_packed_workspace_bytes": (_SZ, [_I, _I, _I]),
    "lp_gemm_update_packed": (_I, [_I, _I, _I, _I, _VP, _I, _VP, _I, _VP, _I, _VP, _SZ, _VP]),
    "lp_ptrans": (_I, [_I, _I, _VP, _I, _VP, _I, _VP, _I, _VP]),
    "lp_convert": (_I, [_I, _I, _I, _VP, _I, _VP, _I, _VP]),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2202_13995_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def _lib() -> ctypes.CDLL:
    """The loaded liblp.so (raises if it is not built; there is no fallback)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def __getattr__(name):
    if name == "lib":
        return _lib()
    raise AttributeError(name)


def strerror(code: int) -> str:
    return _lib().lp_strerror(int(code)).decode()


def _check(fn: str, rc: int) -> None:
    if rc != LP_OK:
        raise LPError(fn, rc)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _keep(t: torch.Tensor, stream) -> None:
    """A tensor allocated here and dropped on return is freed to torch's caching
    allocator on the current stream; when the work was queued on another stream,
    mark it used there so the block is not handed out before that work ends."""
    if stream is not None and t is not None:
        t.record_stream(stream)


def _mat(t: torch.Tensor, dtype=None, name="matrix") -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D row-major with unit column stride")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.stride(0) if t.shape[0] > 0 else max(1, t.shape[1])


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def storage_dtype(prec) -> torch.dtype:
    return torch.float64 if _prec(prec) == FP64 else torch.float32


def workspace(n: int, nb: int, prec="fp64", device="cuda") -> torch.Tensor:
    nbytes = _lib().lu_workspace_bytes(n, nb, _prec(prec))
    if nbytes == 0:
        raise ValueError(f"unsupported (n={n}, nb={nb}, prec={prec})")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def lu_factor(A: torch.Tensor, nb: int, prec="fp64", work=None, ipiv=None, info=None,
              stream=None, lookahead: bool = True, profile: bool = False,
              panel_cus: int = 0, panel_rows: int = 0, pivot: bool = True,
              split_rows: int = 0):
    """In place: A := L\\U. Returns (ipiv int32[n], info int32[1]) on the device, plus a
    per-phase profile dict when profile=True (the call then synchronizes).
    panel_cus / panel_rows: compute units reserved for short panels (see
    lp_factor_opts in include/lp.h; 0 / 0: never).  pivot=False: the no-pivot
    elimination of lu_factor_nopiv (ipiv is then the identity).  split_rows: panels of at
    least this many rows in two halves (lp_factor_opts.panel_split_rows; 0 the default
    choice, -1 never)."""
    p = _prec(prec)
    lda = _mat(A, storage_dtype(p), "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if work is None:
        work = workspace(n, nb, p, A.device)
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    opts = FactorOpts(1 if lookahead else 0, panel_cus, panel_rows, 0 if pivot else 1,
                      split_rows)
    prof = FactorProfile() if profile else None
    _check("lu_factor", _lib().lu_factor_ex(n, nb, p, A.data_ptr(), lda, ipiv.data_ptr(),
                                         info.data_ptr(), work.data_ptr(), work.numel(),
                                         ctypes.byref(opts),
                                         ctypes.byref(prof) if prof is not None else None,
                                         _stream(stream)))
    _keep(work, stream)
    if profile:
        return ipiv, info, prof.as_dict()
    return ipiv, info


def lu_solve(LU: torch.Tensor, ipiv: torch.Tensor, info: torch.Tensor, B: torch.Tensor,
             status=None, stream=None, work=None, persistent: bool = True):
    """In place: B := A^-1 B from the factors. Returns the device solve status.
    persistent=True (default) uses lu_solve_ex, one launch per triangle, with
    `work` (allocated here when None); False uses lu_solve (no workspace)."""
    dt = LU.dtype
    storage = FP64 if dt == torch.float64 else FP32
    lda = _mat(LU, dt, "LU")
    ldb = _mat(B, dt, "B")
    n = LU.shape[0]
    if B.shape[0] != n:
        raise ValueError("B has the wrong number of rows")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=LU.device)
    if not persistent:
        _check("lu_solve", _lib().lu_solve(n, storage, LU.data_ptr(), lda, ipiv.data_ptr(),
                                           info.data_ptr(), B.data_ptr(), ldb, B.shape[1],
                                           status.data_ptr(), _stream(stream)))
        return status
    if work is None:
        work = torch.empty(_lib().lu_solve_workspace_bytes(n, storage, B.shape[1]),
                           dtype=torch.uint8, device=LU.device)
    _check("lu_solve_ex", _lib().lu_solve_ex(n, storage, LU.data_ptr(), lda, ipiv.data_ptr(),
                                             info.data_ptr(), B.data_ptr(), ldb, B.shape[1],
                                             status.data_ptr(), work.data_ptr(), work.numel(),
                                             _stream(stream)))
    _keep(work, stream)
    return status


def residual_check(A: torch.Tensor, X: torch.Tensor, B: torch.Tensor, out=None,
                   stream=None) -> torch.Tensor:
    """Device tensor (nrhs, 5): {s, ||r||, ||A||, ||x||, ||b||} per right-hand side."""
    lda = _mat(A, torch.float64, "A")
    ldx = _mat(X, torch.float64, "X")
    ldb = _mat(B, torch.float64, "B")
    n = A.shape[0]
    nrhs = X.shape[1]
    if out is None:
        out = torch.empty((max(nrhs, 1), 5), dtype=torch.float64, device=A.device)
    _check("residual_check", _lib().residual_check(n, A.data_ptr(), lda, X.data_ptr(), ldx,
                                                B.data_ptr(), ldb, nrhs, out.data_ptr(),
                                                _stream(stream)))
    return out


def solve_ir(A: torch.Tensor, B: torch.Tensor, nb: int, prec="bf16", max_iter: int = 30,
             X=None, work=None, stream=None, gmres: int = 1, gmres_restart: int = 64,
             gmres_max_inner: int = 64, gmres_tol: float = 1e-10, lookahead: bool = True):
    """Mixed-precision solve with binary64 iterative refinement. Returns (X, report).
    gmres: 0 classical corrections only, 1 switch to GMRES corrections when
    classical ones stall (default), 2 GMRES only (lu_solve_ir_ex)."""
    p = _prec(prec)
    lda = _mat(A, torch.float64, "A")
    ldb = _mat(B, torch.float64, "B")
    n, nrhs = B.shape
    if X is None:
        X = torch.empty_like(B)
    ldx = _mat(X, torch.float64, "X")
    if work is None:
        nbytes = _lib().lu_solve_ir_workspace_bytes(n, nb, p, nrhs)
        if nbytes == 0:
            raise ValueError("unsupported solve_ir arguments")
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    rep = IRReport()
    opts = IROpts(max_iter, gmres, gmres_restart, gmres_max_inner, gmres_tol,
                  0 if lookahead else 1)
    _check("lu_solve_ir", _lib().lu_solve_ir_ex(n, nb, p, A.data_ptr(), lda, B.data_ptr(), ldb,
                                                X.data_ptr(), ldx, nrhs, ctypes.byref(opts),
                                                work.data_ptr(), work.numel(), ctypes.byref(rep),
                                                _stream(stream)))
    _keep(work, stream)
    return X, rep


def ir_decide(history, corrections: int, max_iter: int) -> int:
    """The refinement rule of lu_solve_ir (host-only): 0 refine, 1 converged, 2 give up."""
    arr = (ctypes.c_double * max(1, len(history)))(*history)
    return int(_lib().lp_ir_decide(arr, len(history), corrections, max_iter))


class Server:
    """Continuous-batching solve server (liblp.so's lp_server_*).

    submit() takes device tensors A (n x n), B (n x nrhs) and an output X of the
    same shape as B, all float64, and returns a ticket; poll() advances the
    server and returns finished results as dicts.  The tensors of a request are
    kept alive here until its result has been returned.
    """

    def __init__(self, memory_bytes: int, small_n_max: int = 128, max_batch: int = 256,
                 batch_slots: int = 4, batch_workgroups: int = 32, large_slots: int = 4):
        self.cfg = ServerCfg(memory_bytes, small_n_max, max_batch, batch_slots,
                             batch_workgroups, large_slots)
        h = ctypes.c_void_p()
        _check("lp_server_create", _lib().lp_server_create(ctypes.byref(self.cfg),
                                                           ctypes.byref(h)))
        self.h = h
        self._live = {}
        self._buf = (Result * 1024)()

    def _request(self, A, B, X, prec, nb, max_iter) -> Request:
        lda = _mat(A, torch.float64, "A")
        ldb = _mat(B, torch.float64, "B")
        ldx = _mat(X, torch.float64, "X")
        n, nrhs = B.shape
        return Request(A.data_ptr(), B.data_ptr(), X.data_ptr(), lda, ldb, ldx, n, nrhs,
                       _prec(prec), nb, max_iter)

    def footprint(self, A, B, X, prec="fp64", nb: int = 64) -> int:
        req = self._request(A, B, X, prec, nb, 0)
        return int(_lib().lp_request_footprint(ctypes.byref(self.cfg), ctypes.byref(req)))

    def submit(self, A, B, X, prec="fp64", nb: int = 64, max_iter: int = 0,
               stream=None) -> int:
        """Queue a request; it runs after the work already on `stream` (default:
        torch's current stream) that produced A and B."""
        req = self._request(A, B, X, prec, nb, max_iter)
        t = ctypes.c_uint64()
        _check("lp_server_submit", _lib().lp_server_submit(self.h, ctypes.byref(req),
                                                           ctypes.byref(t), _stream(stream)))
        self._live[t.value] = (A, B, X)
        return t.value

    def poll(self) -> list:
        cnt = ctypes.c_int()
        _check("lp_server_poll", _lib().lp_server_poll(self.h, self._buf, len(self._buf),
                                                       ctypes.byref(cnt)))
        out = []
        for i in range(cnt.value):
            d = self._buf[i].as_dict()
            self._live.pop(d["ticket"], None)
            out.append(d)
        return out

    def pending(self):
        q, r, used = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check("lp_server_pending", _lib().lp_server_pending(self.h, ctypes.byref(q),
                                                             ctypes.byref(r),
                                                             ctypes.byref(used)))
        return q.value, r.value, used.value

    def drain(self, timeout_s: float = 120.0) -> list:
        import time
        out = []
        t0 = time.monotonic()
        while self._live:
            got = self.poll()
            out += got
            if not got:
                time.sleep(20e-6)
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
        return out

    def close(self) -> None:
        if self.h:
            _lib().lp_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ------------------------------------------------------------ building blocks
def panel_factor(P: torch.Tensor, prec="fp64", work=None, stream=None, max_wgs: int = 0):
    """Partial-pivoting LU of the column panel P (m x w) in place. Returns (ipiv, info).
    max_wgs > 0 launches at most that many workgroups of up to 1024 rows (the
    shape of panels factored beside the trailing update)."""
    p = _prec(prec)
    ld = _mat(P, storage_dtype(p), "panel")
    m, w = P.shape
    if work is None:
        work = workspace(m, max(w, 1), p, P.device)
    ipiv = torch.empty(max(w, 1), dtype=torch.int32, device=P.device)
    info = torch.empty(1, dtype=torch.int32, device=P.device)
    _check("lp_panel_factor", _lib().lp_panel_factor(m, w, p, P.data_ptr(), ld, ipiv.data_ptr(),
                                                  info.data_ptr(), work.data_ptr(),
                                                  work.numel(), max_wgs, _stream(stream)))
    _keep(work, stream)
    return ipiv, info


def laswp(A: torch.Tensor, c0: int, c1: int, k1: int, k2: int, ipiv: torch.Tensor,
          stream=None) -> None:
    p = FP64 if A.dtype == torch.float64 else FP32
    lda = _mat(A, None, "A")
    nbytes = _lib().lp_laswp_workspace_bytes(k2 - k1)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=A.device)
    _check("lp_laswp", _lib().lp_laswp(p, A.data_ptr(), lda, c0, c1, k1, k2, ipiv.data_ptr(),
                                    work.data_ptr(), work.numel(), _stream(stream)))
    _keep(work, stream)


def trsm_lower_unit(L: torch.Tensor, B: torch.Tensor, stream=None) -> None:
    p = FP64 if B.dtype == torch.float64 else FP32
    ldl = _mat(L, B.dtype, "L")
    ldb = _mat(B, B.dtype, "B")
    m = B.shape[0]
    nbytes = _lib().lp_trsm_workspace_bytes(m)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=B.device)
    _check("lp_trsm_lower_unit", _lib().lp_trsm_lower_unit(p, m, B.shape[1], L.data_ptr(), ldl,
                                                           B.data_ptr(), ldb, work.data_ptr(),
                                                           work.numel(), _stream(stream)))
    _keep(work, stream)


def trsm_right_upper(U: torch.Tensor, B: torch.Tensor, stream=None) -> None:
    """In place: B := B U^-1 with U upper triangular, non-unit (w x w)."""
    p = FP64 if B.dtype == torch.float64 else FP32
    ldu = _mat(U, B.dtype, "U")
    ldb = _mat(B, B.dtype, "B")
    m, w = B.shape
    if U.shape[0] != w or U.shape[1] < w:
        raise ValueError("U must be w x w")
    nbytes = _lib().lp_trsm_right_workspace_bytes(w)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=B.device)
    _check("lp_trsm_right_upper", _lib().lp_trsm_right_upper(p, m, w, U.data_ptr(), ldu,
                                                             B.data_ptr(), ldb, work.data_ptr(),
                                                             work.numel(), _stream(stream)))
    _keep(work, stream)


def lu_factor_nopiv(A: torch.Tensor, nb: int, prec="fp64", work=None, ipiv=None, info=None,
                    stream=None):
    """In place: A := L\\U without row exchanges (lu_factor_nopiv). Returns (ipiv, info)."""
    p = _prec(prec)
    lda = _mat(A, storage_dtype(p), "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if work is None:
        work = workspace(n, nb, p, A.device)
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    _check("lu_factor_nopiv", _lib().lu_factor_nopiv(n, nb, p, A.data_ptr(), lda, ipiv.data_ptr(),
                                                     info.data_ptr(), work.data_ptr(),
                                                     work.numel(), _stream(stream)))
    _keep(work, stream)
    return ipiv, info


def gemm_update(C: torch.Tensor, A: torch.Tensor, B: torch.Tensor, prec=None,
                stream=None) -> None:
    """C := C - A B on the matrix cores (prec defaults to the storage precision)."""
    if prec is None:
        prec = FP64 if C.dtype == torch.float64 else FP32
    p = _prec(prec)
    dt = storage_dtype(p)
    lda = _mat(A, dt, "A")
    ldb = _mat(B, dt, "B")
    ldc = _mat(C, dt, "C")
    M, K = A.shape
    N = B.shape[1]
    if B.shape[0] != K or C.shape != (M, N):
        raise ValueError("shape mismatch")
    _check("lp_gemm_update", _lib().lp_gemm_update(p, M, N, K, A.data_ptr(), lda, B.data_ptr(), ldb,
                                                C.data_ptr(), ldc, _stream(stream)))


def gemm_update_packed(C: torch.Tensor, A: torch.Tensor, B: torch.Tensor, prec=BF16,
                       work=None, stream=None) -> None:
    """C := C - A B (binary32 storage) through packed bfloat16 / half operands."""
    p = _prec(prec)
    lda = _mat(A, torch.float32, "A")
    ldb = _mat(B, torch.float32, "B")
    ldc = _mat(C, torch.float32, "C")
    M, K = A.shape
    N = B.shape[1]
    if B.shape[0] != K or C.shape != (M, N):
        raise ValueError("shape mismatch")
    nbytes = _lib().lp_gemm_packed_workspace_bytes(M, N, K)
    if nbytes == 0:
        raise ValueError("unsupported size")
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=C.device)
    _check("lp_gemm_update_packed",
           _lib().lp_gemm_update_packed(p, M, N, K, A.data_ptr(), lda, B.data_ptr(), ldb,
                                        C.data_ptr(), ldc, work.data_ptr(), work.numel(),
                                        _stream(stream)))
    _keep(work, stream)


def ptrans(A: torch.Tensor, B: torch.Tensor, C=None, stream=None) -> torch.Tensor:
    """C := B + A^T (the paper's PTRANS); C defaults to a new tensor, may be B."""
    dt = A.dtype
    p = FP64 if dt == torch.float64 else FP32
    n = A.shape[0]
    if A.shape != (n, n) or B.shape != (n, n):
        raise ValueError("A and B must be n x n")
    lda = _mat(A, dt, "A")
    ldb = _mat(B, dt, "B")
    if C is None:
        C = torch.empty_like(B)
    ldc = _mat(C, dt, "C")
    _check("lp_ptrans", _lib().lp_ptrans(p, n, A.data_ptr(), lda, B.data_ptr(), ldb, C.data_ptr(),
                                         ldc, _stream(stream)))
    return C


def convert(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    to_f32 = 1 if src.dtype == torch.float64 else 0
    lds = _mat(src, None, "src")
    ldd = _mat(dst, None, "dst")
    _check("lp_convert", _lib().lp_convert(to_f32, src.shape[0], src.shape[1], src.data_ptr(), lds,
                                        dst.data_ptr(), ldd, _stream(stream)))


def flops(n: int, nrhs: int = 1) -> float:
    """LINPACK operation count of factor + solve: 2/3 n^3 + 2 n^2 per right-hand side."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n ** 2 * nrhs
