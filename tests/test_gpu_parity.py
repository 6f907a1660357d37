"""GPU parity: every HIP step against the CPU oracle (or its plain definition).

Run on an MI355X: python -m pytest tests -m gpu.  Inputs come from the seeded
generator in ``inputs`` (host side for the oracle, uploaded unchanged).
Tolerances: binary64 results are compared against bounds derived from the
arithmetic (k * eps * sum of magnitudes for dot products of length k), pivots
and integer outputs bit-exactly.
"""
import numpy as np
import pytest
import scipy.linalg

import inputs
import oracle

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


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


# ------------------------------------------------------------------- inputs
def test_device_generator_matches_host_bitwise(lp):
    import torch
    for n, shift in ((37, 0.0), (300, 300.0), (1024, 0.0)):
        t = torch.empty((n, n), dtype=torch.float64, device="cuda")
        inputs.fill_matrix_(t, 2202, shift=shift)
        a = inputs.matrix(2202, n, shift=shift)
        assert np.array_equal(host(t), a)
    b = torch.empty((100, 3), dtype=torch.float64, device="cuda")
    inputs.fill_rhs_(b, 5)
    assert np.array_equal(host(b), inputs.rhs(5, 100, 3))


# --------------------------------------------------------------------- gemm
@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (1, 1, 1), (17, 33, 5), (128, 128, 16),
                                   (129, 257, 64), (300, 70, 129), (1000, 1000, 64),
                                   (2050, 130, 512)])
def test_gemm_update_f64(lp, M, N, K):
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.uniform(-1, 1, (M, K))
    B = rng.uniform(-1, 1, (K, N))
    C = rng.uniform(-1, 1, (M, N))
    tC = cuda(C)
    lp.gemm_update(tC, cuda(A), cuda(B))
    ref = C - A @ B
    bound = (K + 2) * EPS * (np.abs(C) + np.abs(A) @ np.abs(B))
    assert np.all(np.abs(host(tC) - ref) <= bound)


def test_gemm_update_strided_views(lp):
    # operands as sub-blocks of one row-major matrix, as inside the factorization
    import torch
    rng = np.random.default_rng(1)
    n = 700
    X = rng.uniform(-0.5, 0.5, (n, n))
    t = cuda(X)
    j0, w = 64, 96
    lp.gemm_update(t[j0 + w:, j0 + w:], t[j0 + w:, j0:j0 + w], t[j0:j0 + w, j0 + w:])
    ref = X.copy()
    ref[j0 + w:, j0 + w:] -= X[j0 + w:, j0:j0 + w] @ X[j0:j0 + w, j0 + w:]
    got = host(t)
    assert np.max(np.abs(got - ref)) <= 200 * EPS * w
    # untouched region stays bitwise equal
    assert np.array_equal(got[:j0 + w], X[:j0 + w])
    assert np.array_equal(got[:, :j0 + w], X[:, :j0 + w])


# ---------------------------------------------------------------------- trsm
@pytest.mark.parametrize("m,ncols", [(1, 5), (16, 16), (17, 300), (64, 1000), (256, 333), (200, 7),
                                     (512, 999), (300, 64), (33, 2)])
def test_trsm_lower_unit(lp, m, ncols):
    rng = np.random.default_rng(m + ncols)
    L = np.tril(rng.uniform(-1, 1, (m, m)), -1) + np.eye(m)
    L[np.triu_indices(m, 1)] = 7.0  # garbage above the diagonal must be ignored
    B = rng.uniform(-1, 1, (m, ncols))
    tB = cuda(B)
    lp.trsm_lower_unit(cuda(L), tB)
    ref = scipy.linalg.solve_triangular(np.tril(L, -1) + np.eye(m), B, lower=True,
                                        unit_diagonal=True)
    scale = np.max(np.abs(ref)) + 1
    assert np.max(np.abs(host(tB) - ref)) <= 1e-12 * scale * m


# --------------------------------------------------------------------- laswp
def seq_swaps(a, k1, k2, ipiv, c0, c1):
    a = a.copy()
    for j in range(k1, k2):
        p = ipiv[j]
        if p != j:
            a[[j, p], c0:c1] = a[[p, j], c0:c1]
    return a


@pytest.mark.parametrize("k,nrows,repeat", [(1, 10, False), (7, 50, True), (64, 1000, True),
                                            (512, 4096, True), (512, 600, True),
                                            (1024, 5000, False)])
def test_laswp_matches_sequential_definition(lp, k, nrows, repeat):
    import torch
    rng = np.random.default_rng(k + nrows)
    k1 = 3
    k2 = k1 + k
    ipiv = np.arange(nrows, dtype=np.int32)
    for j in range(k1, k2):
        if repeat and j > k1 and rng.random() < 0.3:
            ipiv[j] = max(j, ipiv[rng.integers(k1, j)])  # revisit an earlier pivot row
        else:
            ipiv[j] = rng.integers(j, nrows)
    ncol = 77
    a = rng.uniform(-1, 1, (nrows, ncol))
    t = cuda(a)
    lp.laswp(t, 5, 70, k1, k2, cuda(ipiv))
    ref = seq_swaps(a, k1, k2, ipiv, 5, 70)
    assert np.array_equal(host(t), ref)


# --------------------------------------------------------------------- panel
@pytest.mark.parametrize("m,w", [(1, 1), (5, 3), (64, 8), (300, 32), (1000, 64), (777, 100),
                                 (5000, 64), (20000, 32), (3000, 256)])
def test_panel_factor_matches_oracle(lp, m, w):
    rng = np.random.default_rng(m * 13 + w)
    P = rng.uniform(-0.5, 0.5, (m, w))
    t = cuda(P)
    ipiv, info = lp.panel_factor(t)
    lu_o, piv_o, info_o = oracle.getrf(P)
    assert int(host(info)[0]) == info_o == 0
    assert np.array_equal(host(ipiv)[:w], piv_o)
    got = host(t)
    assert np.max(np.abs(got - lu_o)) <= 1e-12 * max(1.0, np.max(np.abs(lu_o)))


def test_panel_zero_column_info(lp):
    rng = np.random.default_rng(3)
    P = rng.uniform(-0.5, 0.5, (600, 40))
    P[:, 5] = 0.0
    t = cuda(P)
    ipiv, info = lp.panel_factor(t)
    _, piv_o, info_o = oracle.getrf(P)
    assert int(host(info)[0]) == info_o == 6
    assert np.array_equal(host(ipiv)[:40], piv_o)


# ------------------------------------------------------------ factor + solve
def factor_and_solve(lp, A, B, nb, prec="fp64"):
    import torch
    tA = cuda(A)
    tB = cuda(B)
    ipiv, info = lp.lu_factor(tA, nb, prec)
    st = lp.lu_solve(tA, ipiv, info, tB)
    return tA, ipiv, info, tB, st


@pytest.mark.parametrize("n,nb", [(1, 1), (2, 1), (2, 8), (63, 8), (64, 64), (65, 64), (127, 8),
                                  (300, 32), (1000, 64), (1031, 64), (1024, 1), (777, 100),
                                  (2048, 256)])
def test_lu_factor_solve_matches_oracle(lp, n, nb):
    A = inputs.matrix(11 + n, n)
    B = inputs.rhs(11 + n, n, 3)
    tA, ipiv, info, tB, st = factor_and_solve(lp, A, B, nb)
    lu_o, piv_o, info_o = oracle.getrf(A)
    x_o = oracle.getrs(lu_o, piv_o, B)
    assert int(host(info)[0]) == info_o == 0
    assert int(host(st)[0]) == 0
    assert np.array_equal(host(ipiv)[:n], piv_o)
    x = host(tB)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    res = oracle.residual(A, x, B)
    assert np.all(res[:, 0] < 16)


@pytest.mark.parametrize("n,nrhs", [(700, 11), (640, 17), (901, 9)])
def test_solve_many_right_hand_sides(lp, n, nrhs):
    """More right-hand sides than one pass of the triangular solves takes (8),
    with and without 16-byte-aligned rows of the factors."""
    A = inputs.matrix(5 + n, n)
    B = inputs.rhs(5 + n, n, nrhs)
    tA, ipiv, info, tB, st = factor_and_solve(lp, A, B, 64)
    lu_o, piv_o, _ = oracle.getrf(A)
    x_o = oracle.getrs(lu_o, piv_o, B)
    assert int(host(st)[0]) == 0
    x = host(tB)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    assert np.all(oracle.residual(A, x, B)[:, 0] < 16)


@pytest.mark.parametrize("n,nb", [(4096, 256), (9000, 128)])
def test_reserved_panel_units_match_oracle(lp, n, nb):
    """Every panel after the first on 32 reserved compute units (1024-row
    workgroups with 16-wide leaves once a panel spans more than one), the rest
    of each step on the other units."""
    import torch
    A = inputs.matrix(31 + n, n)
    B = inputs.rhs(31 + n, n, 2)
    tA, tB = cuda(A), cuda(B)
    ipiv, info = lp.lu_factor(tA, nb, "fp64", panel_cus=32, panel_rows=n)
    lp.lu_solve(tA, ipiv, info, tB)
    lu_o, piv_o, info_o = oracle.getrf(A)
    x_o = oracle.getrs(lu_o, piv_o, B)
    assert int(host(info)[0]) == info_o == 0
    assert np.array_equal(host(ipiv)[:n], piv_o)
    x = host(tB)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    assert np.all(oracle.residual(A, x, B)[:, 0] < 16)


def test_config1_parity(lp):
    """n = 1024, nb = 64, A and b uniform[-0.5, 0.5) from seed 2202."""
    import torch
    n, nb, seed = 1024, 64, 2202
    tA = torch.empty((n, n), dtype=torch.float64, device="cuda")
    inputs.fill_matrix_(tA, seed)
    tA0 = tA.clone()
    tB = torch.empty((n, 1), dtype=torch.float64, device="cuda")
    inputs.fill_rhs_(tB, seed)
    tB0 = tB.clone()
    ipiv, info = lp.lu_factor(tA, nb)
    lp.lu_solve(tA, ipiv, info, tB)
    out = host(lp.residual_check(tA0, tB, tB0))
    A = inputs.matrix(seed, n)
    b = inputs.rhs(seed, n, 1)
    lu_o, piv_o, _ = oracle.getrf(A)
    x_o = oracle.getrs(lu_o, piv_o, b)
    assert np.array_equal(host(ipiv)[:n], piv_o)
    x = host(tB)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    ro = oracle.residual(A, x, b)
    assert out[0, 0] < 16 and ro[0, 0] < 16
    # the GPU residual check against the oracle's on the same x
    assert np.allclose(out[0, 2:], ro[0, 2:], rtol=1e-13, atol=0)
    _, absdot = oracle.row_residuals(A, x, b)
    assert abs(out[0, 1] - ro[0, 1]) <= 2 * (n + 2) * EPS * np.max(absdot)


def test_singular_matrix_info_and_solve_refusal(lp):
    n = 200
    A = inputs.matrix(4, n)
    A[:, 17] = 0.0
    B = inputs.rhs(4, n, 2)
    tA, ipiv, info, tB, st = factor_and_solve(lp, A, B, 32)
    _, _, info_o = oracle.getrf(A)
    assert int(host(info)[0]) == info_o == 18
    assert int(host(st)[0]) == 1
    assert np.array_equal(host(tB), B)


def test_diagonally_dominant_identity_pivots(lp):
    n = 1000
    A = inputs.matrix(9, n, shift=float(n))
    B = inputs.rhs(9, n, 1)
    tA, ipiv, info, tB, st = factor_and_solve(lp, A, B, 64)
    assert np.array_equal(host(ipiv)[:n], np.arange(n))
    x_o = oracle.solve(A, B)
    assert np.max(np.abs(host(tB) - x_o)) / np.max(np.abs(x_o)) <= 1e-13


def test_factorization_is_deterministic(lp):
    import torch
    n = 1500
    A = inputs.matrix(21, n)
    outs = []
    for _ in range(2):
        tA = cuda(A)
        ipiv, info = lp.lu_factor(tA, 64)
        outs.append((host(tA), host(ipiv)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("lookahead", [True, False])
def test_factor_profile_accounts_every_step(lp, lookahead):
    """lu_factor_ex's profile: the algorithmic counts follow from n and nb
    alone (sum of 2 M N K over the trailing updates, w^2 N over the "top"
    solves, 32 w N bytes of exchanges right and 32 w j0 left of each panel),
    whichever streams ran the work, and the factors equal those of the same
    call without a profile."""
    n, nb = 4096 + 40, 256
    A = inputs.matrix(17, n)
    t0, t1 = cuda(A), cuda(A)
    ipiv0, _ = lp.lu_factor(t0, nb, lookahead=lookahead)
    ipiv1, info, prof = lp.lu_factor(t1, nb, lookahead=lookahead, profile=True)
    assert int(host(info)[0]) == 0
    assert np.array_equal(host(t0), host(t1)) and np.array_equal(host(ipiv0), host(ipiv1))
    flops = trsm = right = left = 0.0
    launches = 0
    for j0 in range(0, n, nb):
        w = min(nb, n - j0)
        j1 = j0 + w
        m = n - j1
        flops += 2.0 * m * m * w
        trsm += 1.0 * w * w * m
        right += 32.0 * w * m
        left += 32.0 * w * j0
        if m > 0:
            # with look-ahead the next panel's columns and the rest are two updates
            launches += 1 + (1 if lookahead and m > min(nb, m) else 0)
    assert prof["panel_launches"] == -(-n // nb)
    assert prof["gemm_launches"] == launches
    assert prof["gemm_flops"] == flops and prof["trsm_flops"] == trsm
    if lookahead:
        # left exchanges on their own stream, counted apart
        assert prof["swap_bytes"] == right and prof["swap_left_bytes"] == left
        assert prof["swap_left_ms"] > 0
    else:
        assert prof["swap_bytes"] == right + left and prof["swap_left_bytes"] == 0
    for k in ("gemm_ms", "panel_ms", "swap_ms", "trsm_ms"):
        assert prof[k] > 0, k
    assert prof["gemm_ms"] < 1e4 and prof["swap_left_ms"] >= 0


# ------------------------------------------------------------------ residual
def test_residual_check_matches_oracle(lp):
    rng = np.random.default_rng(5)
    n, nrhs = 513, 11
    A = rng.uniform(-0.5, 0.5, (n, n))
    B = rng.uniform(-0.5, 0.5, (n, nrhs))
    X = oracle.solve(A, B)
    out = host(lp.residual_check(cuda(A), cuda(X), cuda(B)))
    ro = oracle.residual(A, X, B)
    _, absdot = oracle.row_residuals(A, X, B)
    assert np.allclose(out[:, 2:], ro[:, 2:], rtol=1e-13, atol=0)
    assert np.all(np.abs(out[:, 1] - ro[:, 1]) <= 2 * (n + 2) * EPS * np.max(absdot, axis=0))
    assert np.all(out[:, 0] < 16)


def test_residual_check_hand_case_and_nan(lp):
    n = 8
    b = np.array([[0.25], [-0.5], [1.0], [0.125], [-2.0], [0.75], [1.5], [-1.0]])
    x = b.copy()
    x[0, 0] += 2.0 ** -20
    out = host(lp.residual_check(cuda(np.eye(n)), cuda(x), cuda(b)))[0]
    assert out[1] == 2.0 ** -20 and out[2] == 1.0 and out[3] == 2.0 and out[4] == 2.0
    assert out[0] == 2.0 ** -20 / (EPS * (2.0 + 2.0) * n)
    a = np.eye(n)
    a[3, 2] = np.nan
    out = host(lp.residual_check(cuda(a), cuda(x), cuda(b)))[0]
    assert not (out[0] < 16)


def test_argument_errors(lp):
    import ctypes
    rc = lp.lib.lu_factor(-1, 64, 0, None, 1, None, None, None, 0, None)
    assert rc == -1
    rc = lp.lib.lu_factor(10, 0, 0, None, 10, None, None, None, 0, None)
    assert rc == -2
    assert lp.lib.lu_workspace_bytes(10, 0, 0) == 0
