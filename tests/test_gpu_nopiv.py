"""GPU parity for the no-pivot LU (the paper's own elimination).

The paper's LINPACK makes A diagonally dominant (the HPL-AI rule) and so
decomposes it without pivoting, per block column: the diagonal block (LU
kernel), the blocks below it with U11 (left), the blocks right of it with L11
(top), the inner blocks with one multiplication.  The GPU path here is
lu_factor_nopiv; the oracle is its unblocked elimination without interchanges
(oracle.getrf_nopiv).  Checked:
  * the right-side upper solve B U^-1 against a host triangular solve
    (entries below U's diagonal are garbage and must not be read);
  * factors against the oracle within 1e-12 (binary64), ipiv the identity,
    x within 1e-10, residual < 16 -- square, ragged and multi-chunk shapes;
  * on A + n I the pivoted path keeps every diagonal row, so both paths
    compute the same factors up to rounding;
  * an exact zero pivot sets info like the oracle;
  * binary32 storage against the oracle on the same binary32 matrix.
"""
import numpy as np
import pytest
import scipy.linalg

import inputs
import oracle

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53
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


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("m,w", [(1, 1), (5, 3), (64, 16), (1000, 64), (777, 100), (300, 128),
                                 (2000, 256), (513, 512), (4099, 200)])
def test_trsm_right_upper(lp, m, w):
    rng = np.random.default_rng(m + 7 * w)
    U = np.triu(rng.uniform(-1, 1, (w, w))) + np.diag(rng.uniform(1, 2, w) * (w ** 0.5))
    Ug = U.copy()
    Ug[np.tril_indices(w, -1)] = 9.0  # below the diagonal: never read
    B = rng.uniform(-1, 1, (m, w))
    tB = cuda(B)
    lp.trsm_right_upper(cuda(Ug), tB)
    ref = scipy.linalg.solve_triangular(U.T, B.T, lower=True).T
    assert rel(host(tB), ref) <= 1e-12


def dominant(seed, n):
    return inputs.matrix(seed, n, shift=float(n))


@pytest.mark.parametrize("n,nb", [(1, 1), (2, 8), (63, 8), (64, 64), (65, 64), (300, 32),
                                  (1000, 64), (1031, 64), (777, 100), (2048, 256), (3000, 512),
                                  (1500, 1024)])
def test_nopiv_matches_oracle(lp, n, nb):
    A = dominant(90 + n, n)
    B = inputs.rhs(90 + n, n, 2)
    tA, tB = cuda(A), cuda(B)
    ipiv, info = lp.lu_factor_nopiv(tA, nb, "fp64")
    st = lp.lu_solve(tA, ipiv, info, tB)
    lu_o, info_o = oracle.getrf_nopiv(A)
    assert int(host(info)[0]) == info_o == 0
    assert int(host(st)[0]) == 0
    assert np.array_equal(host(ipiv)[:n], np.arange(n))
    assert rel(host(tA), lu_o) <= 1e-12
    x_o = oracle.getrs(lu_o, None, B)
    x = host(tB)
    assert rel(x, x_o) <= 1e-10
    assert np.all(oracle.residual(A, x, B)[:, 0] < 16)


@pytest.mark.parametrize("n,nb", [(2048, 256), (4096, 512)])
def test_nopiv_equals_pivoted_on_shifted_matrix(lp, n, nb):
    A = dominant(3, n)
    t1, t2 = cuda(A), cuda(A)
    ipiv1, _ = lp.lu_factor(t1, nb, "fp64")
    ipiv2, _ = lp.lu_factor_nopiv(t2, nb, "fp64")
    assert np.array_equal(host(ipiv1)[:n], np.arange(n))
    assert np.array_equal(host(ipiv2)[:n], np.arange(n))
    assert rel(host(t2), host(t1)) <= 1e-13


def test_nopiv_zero_pivot_info(lp):
    n, k = 200, 37
    A = dominant(8, n)
    A[k, :] = 0.0
    A[:, k] = 0.0
    _, info_o = oracle.getrf_nopiv(A)
    assert info_o == k + 1
    for nb in (16, 32, 64):
        t = cuda(A)
        _, info = lp.lu_factor_nopiv(t, nb, "fp64")
        assert int(host(info)[0]) == k + 1
    A2 = dominant(8, n)
    A2[0, 0] = 0.0
    A2[0, 1:] = 0.0
    _, info = lp.lu_factor_nopiv(cuda(A2), 64, "fp64")
    assert int(host(info)[0]) == 1


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,nb", [(300, 64), (2048, 256)])
def test_nopiv_low_precision_storage(lp, prec, n, nb):
    a32 = dominant(60 + n, n).astype(np.float32)
    t = cuda(a32)
    ipiv, info = lp.lu_factor_nopiv(t, nb, prec)
    lu_o, info_o = oracle.getrf_nopiv(a32.astype(np.float64))
    assert int(host(info)[0]) == info_o == 0
    got = host(t).astype(np.float64)
    if prec == "fp32":
        assert np.max(np.abs(got - lu_o)) <= 200 * n * U32 * np.max(np.abs(lu_o))
    # any rounding of the update operands: A = L U within the backward-error bound
    L = np.tril(got, -1) + np.eye(n)
    U = np.triu(got)
    # binary32 accumulation, plus (bfloat16) one rounding of each update operand
    rnd = 0.0 if prec == "fp32" else 4 * 2.0 ** -8
    bound = (rnd + 4 * n * U32) * (np.abs(L) @ np.abs(U))
    assert np.all(np.abs(a32.astype(np.float64) - L @ U) <= bound)


def test_nopiv_fullsize_shifted_65536(lp):
    """n = 65536, nb = 512 on A + n I: the no-pivot path against the pivoted
    one on the same system (whose pivots must all be diagonal)."""
    import torch
    n, nb, seed = 65536, 512, 2202
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    inputs.fill_matrix_(A0, seed, shift=float(n))
    B = torch.empty((n, 1), dtype=torch.float64, device="cuda")
    inputs.fill_rhs_(B, seed)
    A = A0.clone()
    X = B.clone()
    ipiv, info = lp.lu_factor_nopiv(A, nb, "fp64")
    lp.lu_solve(A, ipiv, info, X)
    out = host(lp.residual_check(A0, X, B))
    assert int(host(info)[0]) == 0 and out[0, 0] < 16
    A2 = A0.clone()
    X2 = B.clone()
    ipiv2, info2 = lp.lu_factor(A2, nb, "fp64")
    lp.lu_solve(A2, ipiv2, info2, X2)
    torch.cuda.synchronize()
    assert torch.equal(ipiv2[:n], torch.arange(n, dtype=torch.int32, device="cuda"))
    d = float((A - A2).abs().max().item()) / float(A2.abs().max().item())
    dx = rel(host(X), host(X2))
    print(f"n={n} shifted: no-pivot vs pivoted factors {d:.2e}, x {dx:.2e}, s {out[0, 0]:.3e}")
    assert d <= 1e-13 and dx <= 1e-13
