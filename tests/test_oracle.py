"""Pins for the CPU oracle (no GPU).

Each test ties the binary64 oracle to something other than itself: exact
rational elimination, closed forms, invariants of partial pivoting, and a
library LU (LAPACK getrf through scipy) on generic inputs.  A dropped term, a
wrong sign or index, a transposed operand, a wrong tie-break or a wrong swap
in the oracle fails at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import brute

EPS = 2.0 ** -53


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def dyadic_matrix(rng, m, n, denom=8, lo=-16, hi=16):
    return rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64) / denom


# ---------------------------------------------------------------- exact, tiny
@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (3, 3), (4, 4), (5, 5), (6, 6),
                                   (6, 3), (5, 2), (3, 5)])
@pytest.mark.parametrize("seed", range(6))
def test_getrf_matches_exact_elimination(shape, seed):
    rng = np.random.default_rng(1000 * seed + shape[0] * 10 + shape[1])
    a = dyadic_matrix(rng, *shape)
    lu_x, piv_x, info_x = brute.getrf_exact(a)
    lu, piv, info = oracle.getrf(a)
    assert list(piv) == piv_x
    assert info == info_x
    exact = np.array([[float(v) for v in row] for row in lu_x])
    scale = max(np.max(np.abs(exact)), 1.0)
    assert np.max(np.abs(lu - exact)) <= 1e-12 * scale


def test_exact_elimination_reconstructs_pa():
    # the rational reference itself: P A = L U exactly
    rng = np.random.default_rng(7)
    for n in range(1, 7):
        a = dyadic_matrix(rng, n, n)
        lu_x, piv_x, info_x = brute.getrf_exact(a)
        assert info_x == 0
        af = brute.to_fractions(a)
        for k, p in enumerate(piv_x):
            af[k], af[p] = af[p], af[k]
        for i in range(n):
            for j in range(n):
                s = sum((lu_x[i][t] if t < i else Fraction(1 if t == i else 0)) * lu_x[t][j]
                        for t in range(min(i, j) + 1) if t <= j)
                assert s == af[i][j]


def test_ties_take_lowest_row_exactly():
    # column 0 holds equal magnitudes with opposite signs: the first row wins
    a = np.array([[1.0, 2.0, 3.0], [-1.0, 5.0, 1.0], [1.0, -2.0, 4.0]])
    lu, piv, info = oracle.getrf(a)
    assert piv[0] == 0
    _, piv_x, _ = brute.getrf_exact(a)
    assert list(piv) == piv_x


def test_exact_inverse_solve_tiny():
    rng = np.random.default_rng(11)
    for n in range(1, 7):
        a = dyadic_matrix(rng, n, n) + n * np.eye(n)
        b = dyadic_matrix(rng, n, 1)[:, 0]
        x_exact = np.array([float(v) for v in brute.solve_exact(a, b)])
        x = oracle.solve(a, b)
        assert rel(x, x_exact) <= 1e-12
        inv = brute.inverse_exact(a)
        af = brute.to_fractions(a)
        for i in range(n):
            for j in range(n):
                assert sum(af[i][t] * inv[t][j] for t in range(n)) == (1 if i == j else 0)


def test_determinant_against_exact():
    rng = np.random.default_rng(5)
    for n in range(2, 9):
        a = dyadic_matrix(rng, n, n)
        lu, piv, info = oracle.getrf(a)
        sign = (-1) ** int(np.sum(piv != np.arange(n)))
        d = sign * np.prod(np.diag(lu))
        dx = float(brute.det_exact(a))
        assert abs(d - dx) <= 1e-12 * max(abs(dx), 1e-3)


# -------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [2, 5, 17, 53])
def test_wilkinson_growth_matrix_bitwise(n):
    a = np.eye(n) - np.tril(np.ones((n, n)), -1)
    a[:, -1] = 1.0
    lu, piv, info = oracle.getrf(a)
    assert info == 0
    assert np.array_equal(piv, np.arange(n))
    L, U = oracle.unpack(lu)
    exp_L = np.eye(n) - np.tril(np.ones((n, n)), -1)
    assert np.array_equal(L, exp_L)
    assert np.array_equal(U[:, -1], 2.0 ** np.arange(n))
    assert np.array_equal(np.diag(U)[:-1], np.ones(n - 1))
    assert np.array_equal(np.triu(U[:, :-1], 1), np.zeros((n, n - 1)))


@pytest.mark.parametrize("n", [1, 4, 33, 100])
def test_permutation_matrix_bitwise(n):
    rng = np.random.default_rng(n)
    perm = rng.permutation(n)
    a = np.eye(n)[perm]
    lu, piv, info = oracle.getrf(a)
    assert info == 0
    L, U = oracle.unpack(lu)
    assert np.array_equal(L, np.eye(n)) and np.array_equal(U, np.eye(n))
    p = oracle.perm_from_ipiv(piv, n)
    assert np.array_equal(a[p], np.eye(n))


@pytest.mark.parametrize("n", [3, 10, 64, 200])
def test_second_difference_matrix_closed_form(n):
    a = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lu, piv, info = oracle.getrf(a)
    assert np.array_equal(piv, np.arange(n))
    k = np.arange(1, n + 1, dtype=np.float64)
    assert rel(np.diag(lu), (k + 1) / k) <= 4 * n * EPS
    assert rel(np.diag(lu, -1), -k[:-1] / (k[:-1] + 1)) <= 4 * n * EPS
    # closed-form inverse: (A^-1)_ij = min(i,j) (n+1-max(i,j)) / (n+1), 1-based
    i = k[:, None]
    j = k[None, :]
    inv = np.minimum(i, j) * (n + 1 - np.maximum(i, j)) / (n + 1)
    x = oracle.getrs(lu, piv, np.eye(n))
    assert rel(x, inv) <= 10 * n * n * EPS


def test_identity_and_diagonal_solve_exact():
    n = 9
    d = np.array([2.0 ** e for e in range(-4, 5)])
    a = np.diag(d)
    b = np.arange(1, n + 1, dtype=np.float64)
    assert np.array_equal(oracle.solve(np.eye(n), b), b)
    assert np.array_equal(oracle.solve(a, b), b / d)


def test_all_ones_construction():
    # the paper builds its input so that the solution is the all-ones vector
    rng = np.random.default_rng(3)
    n = 300
    a = rng.integers(-8, 9, size=(n, n)).astype(np.float64) + 8 * n * np.eye(n)
    b = a.sum(axis=1)          # exact: integers well below 2^53
    x = oracle.solve(a, b)
    assert np.max(np.abs(x - 1.0)) <= 1e-13


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def generic():
    rng = np.random.default_rng(2202)
    n = 257
    a = rng.uniform(-0.5, 0.5, size=(n, n))
    lu, piv, info = oracle.getrf(a)
    return a, lu, piv, info


def test_invariants_pivoting(generic):
    a, lu, piv, info = generic
    n = a.shape[0]
    assert info == 0
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    L, U = oracle.unpack(lu)
    assert np.max(np.abs(np.tril(lu, -1))) <= 1.0
    p = oracle.perm_from_ipiv(piv, n)
    err = np.max(np.sum(np.abs(a[p] - L @ U), axis=1)) / np.max(np.sum(np.abs(a), axis=1))
    assert err <= 8 * n * EPS


def test_power_of_two_scaling_bitwise(generic):
    a, lu, piv, _ = generic
    for s in (-7, 3):
        lu2, piv2, _ = oracle.getrf(a * 2.0 ** s)
        assert np.array_equal(piv2, piv)
        assert np.array_equal(np.tril(lu2, -1), np.tril(lu, -1))
        assert np.array_equal(np.triu(lu2), np.triu(lu) * 2.0 ** s)


def test_row_permutation_keeps_u_bitwise(generic):
    a, lu, piv, _ = generic
    n = a.shape[0]
    q = np.random.default_rng(9).permutation(n)
    lu2, piv2, _ = oracle.getrf(a[q])
    assert np.array_equal(np.triu(lu2), np.triu(lu))


def test_diagonally_dominant_needs_no_pivoting(generic):
    a, _, _, _ = generic
    n = a.shape[0]
    lu, piv, info = oracle.getrf(a + n * np.eye(n))
    assert np.array_equal(piv, np.arange(n))
    lu_np, info_np = oracle.getrf_nopiv(a + n * np.eye(n))
    assert np.array_equal(lu, lu_np)


@pytest.mark.parametrize("n", [64, 500, 1024])
def test_library_lu_cross_check(n):
    rng = np.random.default_rng(n + 1)
    a = rng.uniform(-0.5, 0.5, size=(n, n))
    lu, piv, info = oracle.getrf(a)
    lu_s, piv_s = scipy.linalg.lu_factor(a)
    assert np.array_equal(piv, piv_s)
    assert np.max(np.abs(lu - lu_s)) <= 1e-11 * max(1.0, np.max(np.abs(lu_s)))


def test_rectangular_panel_against_library():
    rng = np.random.default_rng(17)
    a = rng.uniform(-0.5, 0.5, size=(700, 48))
    lu, piv, info = oracle.getrf(a)
    P, L, U = scipy.linalg.lu(a)
    p = oracle.perm_from_ipiv(piv, 700)
    Lo, Uo = oracle.unpack(lu)
    assert np.max(np.abs(Lo @ Uo - a[p])) <= 1e-13
    assert np.allclose(np.abs(np.diag(Uo)), np.abs(np.diag(U)), rtol=1e-12)


# ------------------------------------------------------------ zero pivots
def test_zero_column_sets_info_and_skips():
    rng = np.random.default_rng(4)
    a = dyadic_matrix(rng, 6, 6)
    a[:, 2] = 0.0
    lu, piv, info = oracle.getrf(a)
    _, piv_x, info_x = brute.getrf_exact(a)
    assert info == 3 == info_x
    assert list(piv) == piv_x
    with pytest.raises(ZeroDivisionError):
        oracle.getrs(lu, piv, np.ones(6))


def test_duplicated_row_is_singular():
    rng = np.random.default_rng(6)
    a = dyadic_matrix(rng, 5, 5)
    a[3] = a[1]
    _, _, info = oracle.getrf(a)
    _, _, info_x = brute.getrf_exact(a)
    assert info == info_x and info > 0


# ----------------------------------------------------------------- residual
def test_residual_hand_case():
    n = 8
    b = np.array([0.25, -0.5, 1.0, 0.125, -2.0, 0.75, 1.5, -1.0])
    delta = 2.0 ** -20
    x = b.copy()
    x[0] += delta
    out = oracle.residual(np.eye(n), x, b)[0]
    assert out[1] == delta
    assert out[2] == 1.0
    assert out[3] == 2.0 and out[4] == 2.0
    assert out[0] == delta / (EPS * (1.0 * 2.0 + 2.0) * n)


def test_residual_nan_fails():
    n = 4
    a = np.eye(n)
    a[2, 1] = np.nan
    out = oracle.residual(a, np.ones(n), np.ones(n))[0]
    assert not (out[0] < 16.0)


def test_residual_long_double_cross_check():
    rng = np.random.default_rng(2)
    n = 400
    a = rng.uniform(-0.5, 0.5, size=(n, n))
    b = rng.uniform(-0.5, 0.5, size=(n, 2))
    x = oracle.solve(a, b)
    r64 = oracle.residual(a, x, b)
    rld = oracle.residual(a, x, b, long_double=True)
    assert np.all(r64[:, 0] < 16) and np.all(rld[:, 0] < 16)
    # norms agree to rounding; ||r|| agrees within the binary64 evaluation bound
    assert np.allclose(r64[:, 2:], rld[:, 2:], rtol=1e-13, atol=0)
    _, absdot = oracle.row_residuals(a, x, b)
    bound = (n + 1) * EPS * np.max(absdot, axis=0) / (1 - (n + 1) * EPS)
    assert np.all(np.abs(r64[:, 1] - rld[:, 1]) <= bound)


def test_row_residuals_match_full():
    rng = np.random.default_rng(8)
    n = 50
    a = rng.uniform(-0.5, 0.5, size=(n, n))
    b = rng.uniform(-0.5, 0.5, size=(n, 3))
    x = oracle.solve(a, b)
    r, _ = oracle.row_residuals(a, x, b)
    full = oracle.residual(a, x, b)
    assert np.allclose(np.max(np.abs(r), axis=0), full[:, 1], rtol=0, atol=0)


# ------------------------------------------- scaling divides (reading: divide)
def test_multipliers_are_correctly_rounded_quotients():
    # The first column's multipliers are a single rounding of a_i0 / a_00.  A
    # correctly rounded division gives float(Fraction(a_i0) / Fraction(a_00))
    # exactly; multiplying by a rounded reciprocal does not (3 * (1/5) is
    # 0.6000000000000001, while 3/5 rounds to 0.6).
    a = np.array([[5.0, 1.0], [3.0, 2.0]])
    lu, piv, info = oracle.getrf(a)
    assert list(piv) == [0, 1] and info == 0
    assert lu[1, 0] == float(Fraction(3, 5))
    assert lu[1, 0] != 3.0 * (1.0 / 5.0)
    # a whole column: pivot 10 (largest), many quotients where the two differ
    col = np.array([10.0] + [float(v) for v in range(1, 10)] + [-3.0, 7.0, -9.0, 9.5])
    a = col.reshape(-1, 1).copy()  # one column: one elimination step
    for getrf in (lambda x: oracle.getrf(x)[0], lambda x: oracle.getrf_nopiv(x)[0]):
        lu = getrf(a)
        exact = [float(Fraction(v) / Fraction(10.0)) for v in col[1:]]
        assert list(lu[1:, 0]) == exact
    recip = col[1:] * (1.0 / 10.0)
    assert np.count_nonzero(recip != np.array(exact)) >= 3


# ------------------------------------------------- transposed solve, estimate
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_transposed_solve_matches_exact(n):
    rng = np.random.default_rng(300 + n)
    a = dyadic_matrix(rng, n, n)
    lu_x, piv_x, info_x = brute.getrf_exact(a)
    if info_x != 0:
        a = a + n * np.eye(n)
    b = dyadic_matrix(rng, n, 1)[:, 0]
    x_exact = np.array([float(v) for v in brute.solve_exact(a.T.copy(), b)])
    lu, piv, info = oracle.getrf(a)
    x = oracle.getrs(lu, piv, b, trans=True)
    assert rel(x, x_exact) <= 1e-12


def test_transposed_solve_generic():
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.5, 0.5, (200, 200))
    b = rng.uniform(-0.5, 0.5, (200, 3))
    lu, piv, _ = oracle.getrf(a)
    x = oracle.getrs(lu, piv, b, trans=True)
    assert rel(a.T @ x, b) <= 1e-11
    assert rel(x, np.linalg.solve(a.T, b)) <= 1e-10


def test_condition_estimate_exact_cases():
    from oracle import cond
    # diagonal: ||A^-1||_inf = max 1/|d_i|, found exactly
    d = np.array([4.0, -0.5, 2.0, 8.0, -0.25])
    lu, piv, _ = oracle.getrf(np.diag(d))
    assert cond.inv_norm_inf_estimate(lu, piv) == 4.0
    # second difference matrix: closed-form inverse min(i,j)(n+1-max(i,j))/(n+1)
    for n in (7, 40, 101):
        a = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        i = np.arange(1, n + 1)
        inv = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
        exact = np.abs(inv).sum(axis=1).max()
        lu, piv, _ = oracle.getrf(a)
        assert abs(cond.inv_norm_inf_estimate(lu, piv) - exact) <= 1e-12 * exact


def test_condition_estimate_is_a_lower_bound():
    from oracle import cond
    import inputs
    hits = 0
    for seed in range(1, 9):
        a = inputs.matrix(seed, 120)
        lu, piv, _ = oracle.getrf(a)
        est = cond.inv_norm_inf_estimate(lu, piv)
        exact = np.abs(np.linalg.inv(a)).sum(axis=1).max()
        assert est <= exact * (1 + 1e-10)
        assert est >= exact / 3
        hits += abs(est - exact) <= 1e-10 * exact
    assert hits >= 6


# ------------------------------------------------------------------ PTRANS
def test_ptrans_special_cases():
    # C = B + A^T (paper, section "Parallel Matrix Transposition")
    rng = np.random.default_rng(12)
    for n in (1, 2, 7, 64, 65, 130):
        a = rng.uniform(-1, 1, (n, n))
        b = rng.uniform(-1, 1, (n, n))
        # B = 0: the plain transpose, bit for bit
        assert np.array_equal(oracle.ptrans(a, np.zeros((n, n))), a.T)
        # A = I: B plus the identity
        assert np.array_equal(oracle.ptrans(np.eye(n), b), b + np.eye(n))
        # symmetric A: the transpose changes nothing
        s = a + a.T
        assert np.array_equal(oracle.ptrans(s, b), b + s)
        # an asymmetric single entry lands transposed
        e = np.zeros((n, n))
        e[n - 1, 0] = 3.0
        c = oracle.ptrans(e, np.zeros((n, n)))
        assert c[0, n - 1] == 3.0 and np.count_nonzero(c) == 1


def test_ptrans_binary32_rounds_once():
    rng = np.random.default_rng(13)
    a = rng.uniform(-1, 1, (50, 50)).astype(np.float32)
    b = rng.uniform(-1, 1, (50, 50)).astype(np.float32)
    c = oracle.ptrans(a, b)
    assert c.dtype == np.float32
    # the exact sum rounded once to binary32
    exact = b.astype(np.float64) + a.T.astype(np.float64)
    assert np.array_equal(c, exact.astype(np.float32))
