"""GPU parity of the split panel (lp_factor_opts.panel_split_rows; by default
the panels of the bfloat16 / half factorizations are split, binary64 and
binary32 panels only when they have at most 8192 rows).  With partial pivoting (paper, section "High
Performance Linpack"), a panel of 256 columns or more is factored as two
halves, the right half brought up to date by one product on the GEMM kernel
between them; only the grouping of the right half's updates changes, never a
pivot decision rule.  Both forms are compared with the oracle's unblocked
elimination:

  * random matrices: pivots bit for bit, x within 1e-10, and every factor
    element within 4 n u (|L||U|)_ij of the oracle's (a bound on any order of
    the same sums);
  * planted matrices P = Pi (L U) with dyadic L (|l| <= 1/2 off the diagonal)
    and small-integer U: every quantity of the elimination, including the
    16x16 block inverses of the triangular solves, is exact in binary64, so
    pivots and factors must equal the oracle's bit for bit, with and without
    the split (in binary32 those block inverses round, so planted matrices
    prove nothing there);
  * binary32 storage on random matrices: pivots agree with the oracle's
    elimination of the same binary32 matrix (near-ties aside), |l| <= 1 and
    P A = L U within the binary32 backward-error bound 4 n u32 |L||U|.
"""
import functools

import numpy as np
import pytest

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


@functools.lru_cache(maxsize=None)
def random_case(n):
    A = inputs.matrix(500 + n, n)
    B = inputs.rhs(500 + n, n, 2)
    lu_o, piv_o, info_o = oracle.getrf(A)
    return A, B, lu_o, piv_o, info_o, oracle.getrs(lu_o, piv_o, B)


@functools.lru_cache(maxsize=None)
def oracle_fp32(n):
    return oracle.getrf(random_case(n)[0].astype(np.float32).astype(np.float64))


@functools.lru_cache(maxsize=None)
def planted_case(seed, n):
    P = planted(seed, n)
    lu_o, piv_o, info_o = oracle.getrf(P)
    return P, lu_o, piv_o, info_o


def planted(seed, n):
    rng = np.random.default_rng(seed)
    L = rng.choice(np.array([0.0, 0.125, -0.125, 0.25, -0.25, 0.5, -0.5]), size=(n, n))
    L = np.tril(L, -1) + np.eye(n)
    U = np.triu(rng.integers(-64, 65, size=(n, n)).astype(np.float64), 1)
    U += np.diag(rng.integers(1, 65, size=n) * rng.choice([-1.0, 1.0], size=n))
    P = L @ U
    assert np.max(np.abs(P)) < 2.0 ** 16
    return P[rng.permutation(n)]


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("n,nb", [(2304, 256), (2560, 512), (2100, 300), (1000, 512)])
def test_split_panels_random_match_oracle(lp, n, nb, split):
    print(f"random n={n} nb={nb} split={split}", flush=True)
    A, B, lu_o, piv_o, info_o, x_o = random_case(n)
    tA = cuda(A)
    ipiv, info = lp.lu_factor(tA, nb, split_rows=(1 if split else -1))
    tB = cuda(B)
    st = lp.lu_solve(tA, ipiv, info, tB)
    assert int(host(info)[0]) == info_o == 0
    assert int(host(st)[0]) == 0
    assert np.array_equal(host(ipiv)[:n], piv_o)
    F = host(tA)
    Lo = np.tril(lu_o, -1) + np.eye(n)
    Uo = np.triu(lu_o)
    bound = 4 * n * EPS * (np.abs(Lo) @ np.abs(Uo))
    assert np.all(np.abs(F - lu_o) <= bound), float(np.max(np.abs(F - lu_o) / bound))
    x = host(tB)
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10


@pytest.mark.parametrize("n,nb", [(2048, 512), (2048, 256), (1800, 320), (1000, 256)])
def test_split_panels_planted_bit_exact(lp, n, nb):
    print(f"planted n={n} nb={nb}", flush=True)
    P, lu_o, piv_o, info_o = planted_case(11, n)
    assert info_o == 0
    for split in (True, False):
        tA = cuda(P)
        ipiv, info = lp.lu_factor(tA, nb, "fp64", split_rows=(1 if split else -1))
        assert int(host(info)[0]) == 0
        assert np.array_equal(host(ipiv)[:n], piv_o), split
        assert np.array_equal(host(tA), lu_o), split


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("n,nb", [(2304, 256), (2560, 512)])
def test_split_panels_binary32(lp, n, nb, split):
    print(f"binary32 n={n} nb={nb} split={split}", flush=True)
    a32 = random_case(n)[0].astype(np.float32)
    lu_o, piv_o, info_o = oracle_fp32(n)
    tA = cuda(a32)
    ipiv, info = lp.lu_factor(tA, nb, "fp32", split_rows=(1 if split else -1))
    assert int(host(info)[0]) == info_o == 0
    got_piv = host(ipiv)[:n]
    assert np.mean(got_piv == piv_o) >= 0.99
    got = host(tA).astype(np.float64)
    assert np.max(np.abs(np.tril(got, -1))) <= 1.0
    L = np.tril(got, -1) + np.eye(n)
    U = np.triu(got)
    pa = a32.astype(np.float64)[oracle.perm_from_ipiv(got_piv, n)]
    assert np.all(np.abs(pa - L @ U) <= 4 * n * 2.0 ** -24 * (np.abs(L) @ np.abs(U)))


@pytest.mark.parametrize("zero_col", [40, 300, 450])
def test_split_panels_first_zero_pivot(lp, zero_col):
    """An exactly singular matrix (one zero column): the split and the single
    launch report the oracle's first zero pivot (info = column + 1)."""
    n, nb = 640, 256
    A = inputs.matrix(23, n)
    A[:, zero_col] = 0.0
    _, _, info_o = oracle.getrf(A)
    assert info_o == zero_col + 1
    for split in (True, False):
        tA = cuda(A)
        _, info = lp.lu_factor(tA, nb, "fp64", split_rows=(1 if split else -1))
        assert int(host(info)[0]) == info_o, split
