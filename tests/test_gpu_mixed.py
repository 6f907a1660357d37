"""GPU parity for the low-precision factorization and iterative refinement.

The binary32 trailing update is checked element-wise against binary64 products
of the same rounded operands (bfloat16 / half rounding from the reference in
oracle/ir.py), the binary32 factorization against the oracle's factorization of
the same binary32 matrix, and the refined solution against the binary64
oracle's solution (scaled residual < 16 and the forward error bound).
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import ir

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2202_13995_amd as lp
    return lp


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("M,N,K", [(16, 16, 32), (1, 1, 1), (130, 70, 33), (300, 257, 64),
                                   (1000, 1000, 256), (2050, 130, 512), (384, 256, 96),
                                   (640, 384, 1024)])
def test_gemm_update_low_precision(lp, prec, M, N, K):
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.uniform(-1, 1, (M, K)).astype(np.float32)
    B = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    C = rng.uniform(-1, 1, (M, N)).astype(np.float32)
    tC = cuda(C)
    lp.gemm_update(tC, cuda(A), cuda(B), prec=prec)
    Ar = ir.round_to(A, prec).astype(np.float64)
    Br = ir.round_to(B, prec).astype(np.float64)
    ref = C.astype(np.float64) - Ar @ Br
    bound = (K + 2) * U32 * (np.abs(C) + np.abs(Ar) @ np.abs(Br)) + 1e-30
    err = np.abs(host(tC).astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (256, 256, 64), (300, 257, 64), (513, 700, 96),
                                   (1000, 1000, 512), (2050, 130, 1024), (700, 2300, 33)])
def test_gemm_update_packed(lp, prec, M, N, K):
    """Packed -A / B^T operands on 256 x 256 tiles: ragged tiles, k padded to a
    power-of-two multiple of 64, strided C; same bound as the unpacked update."""
    rng = np.random.default_rng(M + 5 * N + 11 * K)
    A = rng.uniform(-1, 1, (M, K + 3)).astype(np.float32)[:, :K]
    B = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    Cfull = rng.uniform(-1, 1, (M, N + 5)).astype(np.float32)
    tA = cuda(np.ascontiguousarray(rng.uniform(-1, 1, (M, K + 3)).astype(np.float32)))
    tA[:, :K] = cuda(A)
    tCf = cuda(Cfull)
    tC = tCf[:, :N]
    lp.gemm_update_packed(tC, tA[:, :K], cuda(B), prec=prec)
    Ar = ir.round_to(A, prec).astype(np.float64)
    Br = ir.round_to(B, prec).astype(np.float64)
    C = Cfull[:, :N]
    ref = C.astype(np.float64) - Ar @ Br
    bound = (K + 2) * U32 * (np.abs(C) + np.abs(Ar) @ np.abs(Br)) + 1e-30
    out = host(tCf)
    err = np.abs(out[:, :N].astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.array_equal(out[:, N:], Cfull[:, N:])  # columns past N untouched


@pytest.mark.parametrize("n,nb", [(64, 32), (300, 64), (1000, 128), (2048, 256)])
def test_fp32_factorization_matches_oracle_on_fp32_matrix(lp, n, nb):
    a32 = inputs.matrix(40 + n, n).astype(np.float32)
    tA = cuda(a32)
    ipiv, info = lp.lu_factor(tA, nb, "fp32")
    lu_o, piv_o, info_o = oracle.getrf(a32.astype(np.float64))
    assert int(host(info)[0]) == info_o == 0
    got_piv = host(ipiv)[:n]
    agree = np.mean(got_piv == piv_o)
    assert agree >= 0.99, agree          # binary32 near-ties may legitimately differ
    got = host(tA).astype(np.float64)
    if agree == 1.0:
        assert np.max(np.abs(got - lu_o)) <= 200 * n * U32
    # whatever the pivots: |l| <= 1 and P A = L U within the binary32
    # backward-error bound of Gaussian elimination (gamma_n |L| |U|)
    assert np.max(np.abs(np.tril(got, -1))) <= 1.0
    L = np.tril(got, -1) + np.eye(n)
    U = np.triu(got)
    pa = a32.astype(np.float64)[oracle.perm_from_ipiv(got_piv, n)]
    bound = 4 * n * U32 * (np.abs(L) @ np.abs(U))
    assert np.all(np.abs(pa - L @ U) <= bound)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_refinement_shifted_matrix(lp, prec):
    import torch
    n, nb = 1024, 128
    A = inputs.matrix(2202, n, shift=float(n))
    B = inputs.rhs(2202, n, 2)
    tA, tB = cuda(A), cuda(B)
    X, rep = lp.solve_ir(tA, tB, nb, prec)
    r = rep.as_dict()
    assert r["converged"] == 1 and r["fell_back"] == 0, r
    assert r["scaled_residual"] < 16 and r["iterations"] <= 6, r
    x = host(X)
    x_o = oracle.solve(A, B)
    # refinement stops at scaled residual < 16, which bounds the forward error by
    # ~cond * 16 * n * eps; the stated tolerance is 1e-10
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    res = oracle.residual(A, x, B)
    assert np.all(res[:, 0] < 16)
    # inputs untouched
    assert np.array_equal(host(tA), A) and np.array_equal(host(tB), B)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_refinement_packed_trailing_updates(lp, prec):
    # n = 6144, nb = 256: the trailing updates right of the next panel run on
    # packed 256 x 256 tiles (with a ragged last tile row and column)
    n, nb = 6144 + 40, 256
    A = inputs.matrix(31, n, shift=float(n))
    B = inputs.rhs(31, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, prec)
    r = rep.as_dict()
    assert r["converged"] == 1 and r["fell_back"] == 0 and r["iterations"] <= 6, r
    x_o = oracle.solve(A, B)
    assert np.max(np.abs(host(X) - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    assert np.all(oracle.residual(A, host(X), B)[:, 0] < 16)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_refinement_unshifted_matrix(lp, prec):
    n, nb = 1000, 64
    A = inputs.matrix(77, n)
    B = inputs.rhs(77, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, prec)
    r = rep.as_dict()
    assert r["scaled_residual"] < 16, r
    x = host(X)
    x_o = oracle.solve(A, B)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    if prec == "fp32":
        assert r["converged"] == 1 and r["fell_back"] == 0 and r["iterations"] <= 4, r


def test_refinement_fallback_recorded(lp):
    # max_iter = 0 forbids corrections: unless x0 already passes, the FP64 path runs
    n = 512
    A = inputs.matrix(9, n)
    B = inputs.rhs(9, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), 64, "bf16", max_iter=0)
    r = rep.as_dict()
    assert r["fell_back"] == 1 and r["converged"] == 1, r
    x_o = oracle.solve(A, B)
    assert np.max(np.abs(host(X) - x_o)) / np.max(np.abs(x_o)) <= 1e-10


def test_refinement_singular_low_precision_falls_back_and_reports(lp):
    n = 256
    A = inputs.matrix(5, n)
    A[:, 10] = 0.0
    B = inputs.rhs(5, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), 64, "fp32")
    r = rep.as_dict()
    assert r["info"] == 11 and r["fell_back"] == 1 and r["fallback_info"] == 11
    assert r["converged"] == 0


def test_fp64_through_refinement_entry(lp):
    n = 300
    A = inputs.matrix(12, n)
    B = inputs.rhs(12, n, 3)
    X, rep = lp.solve_ir(cuda(A), cuda(B), 64, "fp64")
    r = rep.as_dict()
    assert r["converged"] == 1 and r["fell_back"] == 0 and r["iterations"] == 0
    x_o = oracle.solve(A, B)
    assert np.max(np.abs(host(X) - x_o)) / np.max(np.abs(x_o)) <= 1e-10


# ------------------------------------------------------------------ GMRES-IR
@pytest.mark.parametrize("n,nb,nrhs", [(2048, 256, 1), (1500, 128, 3)])
def test_gmres_refinement_unshifted(lp, n, nb, nrhs):
    """GMRES corrections only (gmres=2) on an unshifted matrix with bfloat16
    factors: converges without the binary64 fallback; x against the oracle."""
    A = inputs.matrix(81 + n, n)
    B = inputs.rhs(81 + n, n, nrhs)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, "bf16", gmres=2, gmres_max_inner=200)
    r = rep.as_dict()
    print(f"GMRES-IR n={n}: {r['iterations']} corrections, {r['gmres_steps']} GMRES steps, "
          f"history {r['history']}")
    assert r["converged"] == 1 and r["fell_back"] == 0, r
    assert r["gmres_corrections"] == r["iterations"] >= 1 and r["gmres_steps"] >= 1
    x_o = oracle.solve(A, B)
    x = host(X)
    assert np.all(oracle.residual(A, x, B)[:, 0] < 16)
    # refinement stops at the benchmark's s < 16, a backward-error criterion:
    # the forward error is bounded by about kappa * s * n * u, not by 1e-10
    kappa = np.linalg.cond(A, np.inf)
    err = np.max(np.abs(x - x_o)) / np.max(np.abs(x_o))
    print(f"forward error {err:.2e}, kappa_inf {kappa:.2e}")
    assert err <= 4 * kappa * max(r["scaled_residual"], 1.0) * n * 2.0 ** -53


def test_gmres_switch_after_classical_stall(lp):
    """Default mode: classical corrections until one fails to cut the residual
    fourfold, then GMRES; the switch is visible in the history."""
    n, nb = 4096, 256
    A = inputs.matrix(5, n)
    B = inputs.rhs(5, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, "bf16", gmres_max_inner=200)
    r = rep.as_dict()
    h = r["history"]
    print(f"n={n} default refinement: history {h}, gmres corrections {r['gmres_corrections']}")
    assert r["converged"] == 1 and r["fell_back"] == 0, r
    ncl = r["iterations"] - r["gmres_corrections"]
    # every classical correction but the last cut the residual fourfold
    for i in range(1, ncl):
        assert h[i] <= 0.25 * h[i - 1]
    if r["gmres_corrections"]:
        assert not (h[ncl] <= 0.25 * h[ncl - 1]) if ncl >= 1 else True
    # stopping at s < 16 bounds the forward error by about kappa * s * n * u
    x_o = oracle.solve(A, B)
    kappa = np.linalg.cond(A, np.inf)
    err = np.max(np.abs(host(X) - x_o)) / np.max(np.abs(x_o))
    print(f"forward error {err:.2e}, kappa_inf {kappa:.2e}")
    assert err <= 4 * kappa * max(r["scaled_residual"], 1.0) * n * 2.0 ** -53


def test_gmres_refinement_is_deterministic(lp):
    n, nb = 1200, 128
    A = inputs.matrix(17, n)
    B = inputs.rhs(17, n, 2)
    xs = []
    for _ in range(2):
        X, rep = lp.solve_ir(cuda(A), cuda(B), nb, "bf16", gmres=2, gmres_max_inner=200)
        xs.append(host(X))
    assert np.array_equal(xs[0], xs[1])


def test_classical_only_mode(lp):
    n, nb = 1000, 64
    A = inputs.matrix(77, n)
    B = inputs.rhs(77, n, 1)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, "bf16", gmres=0)
    r = rep.as_dict()
    assert r["gmres_corrections"] == 0 and r["gmres_steps"] == 0
    assert r["scaled_residual"] < 16


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_refinement_without_lookahead(lp, prec):
    """lp_ir_opts.no_lookahead runs the factorization's steps in order on one
    stream.  In binary32 every element sees the same operations in the same
    order, so x, the history and the decisions are bitwise the same; with
    bfloat16 operands the next panel's columns may take the unpacked update
    kernel under look-ahead, so there both must converge to the same x within
    the refinement's accuracy."""
    n, nb = 1536, 128
    A = inputs.matrix(91, n, shift=float(n))
    B = inputs.rhs(91, n, 2)
    out = []
    for la in (True, False):
        X, rep = lp.solve_ir(cuda(A), cuda(B), nb, prec, lookahead=la)
        r = rep.as_dict()
        out.append((host(X), r["history"], r["iterations"], r["fell_back"]))
    for x, hist, _, fb in out:
        assert hist[-1] < 16 and fb == 0
    if prec == "fp32":
        assert np.array_equal(out[0][0], out[1][0])
        assert out[0][1:] == out[1][1:]
    else:
        d = np.max(np.abs(out[0][0] - out[1][0])) / np.max(np.abs(out[1][0]))
        assert d <= 1e-10, d


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_refinement_block_1024(lp, prec):
    """A 1024-wide block (the bfloat16 benchmark's): each panel is factored in
    quarters, split twice, with GEMM-kernel updates between them; the refined
    x must still pass the binary64 scaled-residual check."""
    n, nb = 4096, 1024
    A = inputs.matrix(123, n, shift=float(n))
    B = inputs.rhs(123, n, 2)
    X, rep = lp.solve_ir(cuda(A), cuda(B), nb, prec)
    r = rep.as_dict()
    assert r["converged"] == 1 and r["fell_back"] == 0, r
    assert np.all(oracle.residual(A, host(X), B)[:, 0] < 16)
