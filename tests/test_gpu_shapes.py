"""GPU parity in the launch shapes the factorization uses at full size.

Inside lu_factor a panel factored beside the trailing update runs on a capped
number of workgroups of up to 1024 rows each (binary64: max(48, ceil(m/1024))
workgroups, 4 row chunks per thread, 16-wide leaves; binary32: max(128, ...),
512 rows per workgroup at m = 65536).  These tests launch exactly those shapes
through lp_panel_factor(max_wgs) on full-size panels and compare them with the
oracle's unblocked elimination of the same panel:

  * random panels (uniform[-0.5, 0.5)): pivots bit-exact, factors within
    1e-12 (binary64);
  * planted panels P = Pi (L U) with dyadic L (|l| <= 1/2, three fractional
    bits) and small-integer U: every quantity of the elimination is exact in
    binary32 and binary64 whatever the summation order, so pivots AND factors
    must equal the oracle's bit for bit in either precision -- this checks the
    pivot search, the row exchanges and the data movement of every shape
    exactly, binary32 included.

Also here: leading dimensions larger than the matrix, with NaN in the padding
(it must be neither read into results nor written).
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


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


def random_panel(seed, m, w):
    idx = (np.arange(m, dtype=np.uint64)[:, None] * np.uint64(w)
           + np.arange(w, dtype=np.uint64)[None, :])
    return inputs.uniform(seed, inputs.STREAM_A, idx)


def planted_panel(seed, m, w):
    """Pi (L U): L m x w unit lower with entries in {0, +-1/8, +-1/4, +-1/2},
    U w x w upper with integers in [-64, 64] and a nonzero diagonal, rows
    shuffled.  Partial sums stay below 2^15 in steps of 1/8 (18 bits)."""
    rng = np.random.default_rng(seed)
    L = rng.choice(np.array([0.0, 0.125, -0.125, 0.25, -0.25, 0.5, -0.5]), size=(m, w))
    L[:w] = np.tril(L[:w], -1) + np.eye(w)
    U = np.triu(rng.integers(-64, 65, size=(w, w)).astype(np.float64), 1)
    d = rng.integers(1, 65, size=w) * rng.choice([-1.0, 1.0], size=w)
    U += np.diag(d)
    P = L @ U
    assert np.max(np.abs(P)) < 2.0 ** 15
    return P[rng.permutation(m)]


# (rows, width, precision, workgroup cap): the shapes lu_factor launches beside
# the trailing update at n = 32768 / nb = 256 (binary64: 48 workgroups of 704
# rows) and n = 65536 / nb = 512 (binary64: 64 of 1024 rows; binary32: 128 of
# 512 rows), a binary32 panel of 256 rows per workgroup, binary64 panels of
# 256 and 512 rows per workgroup with 32-wide leaves, and whole-device panels
# (cap 0: one workgroup per 256 rows, 254 workgroups here).
SHAPES = [(32512, 256, "fp64", 48), (65024, 512, "fp64", 64),
          (65024, 512, "fp32", 128), (32000, 512, "fp32", 128),
          (12288, 512, "fp64", 48), (24000, 256, "fp64", 48),
          (65024, 512, "fp64", 0), (65024, 256, "fp32", 0)]


@pytest.mark.parametrize("m,w,prec,wgs", SHAPES)
def test_planted_panel_bit_exact(lp, m, w, prec, wgs):
    P = planted_panel(m + w, m, w)
    lu_o, piv_o, info_o = oracle.getrf(P)
    assert info_o == 0
    dt = np.float64 if prec == "fp64" else np.float32
    t = cuda(P.astype(dt))
    print(f"planted panel {m}x{w} {prec} max_wgs={wgs}", flush=True)
    ipiv, info = lp.panel_factor(t, prec, max_wgs=wgs)
    assert int(host(info)[0]) == 0
    assert np.array_equal(host(ipiv)[:w], piv_o)
    assert np.array_equal(host(t).astype(np.float64), lu_o)


@pytest.mark.parametrize("m,w,wgs", [(32512, 256, 48), (65024, 512, 64), (24576 + 700, 256, 48)])
def test_random_panel_fullsize_shape_fp64(lp, m, w, wgs):
    P = random_panel(2202 + m, m, w)
    lu_o, piv_o, info_o = oracle.getrf(P)
    t = cuda(P)
    print(f"random panel {m}x{w} fp64 max_wgs={wgs}", flush=True)
    ipiv, info = lp.panel_factor(t, "fp64", max_wgs=wgs)
    assert int(host(info)[0]) == info_o == 0
    assert np.array_equal(host(ipiv)[:w], piv_o)
    got = host(t)
    assert np.max(np.abs(got - lu_o)) <= 1e-12 * max(1.0, np.max(np.abs(lu_o)))
    assert np.max(np.abs(np.tril(got, -1))) <= 1.0


def test_random_panel_fp32_128_workgroups(lp):
    """A binary32 panel in the 128-workgroup shape: |l| <= 1 exactly, pivots
    agree with the binary64 oracle on the same binary32 data except where
    binary32 rounding legitimately reorders near ties (reported), and the
    factors reproduce P A within the binary32 backward-error bound on sampled
    entries."""
    m, w = 65024, 512
    P = random_panel(7, m, w).astype(np.float32)
    t = cuda(P)
    ipiv, info = lp.panel_factor(t, "fp32", max_wgs=128)
    got = host(t).astype(np.float64)
    piv = host(ipiv)[:w].astype(np.int64)
    assert int(host(info)[0]) == 0
    assert np.all(piv >= np.arange(w)) and np.all(piv < m)
    assert np.max(np.abs(np.tril(got, -1))) <= 1.0
    _, piv_o, _ = oracle.getrf(P.astype(np.float64))
    first = int(np.argmax(piv != piv_o)) if np.any(piv != piv_o) else w
    print(f"binary32 panel: pivots equal to the oracle's for the first {first} of {w} columns,"
          f" {np.mean(piv == piv_o):.3f} of all")
    perm = oracle.perm_from_ipiv(piv, m)
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([np.arange(w), rng.integers(w, m, 256)]))
    L = np.where(np.arange(w)[None, :] < rows[:, None], got[rows], 0.0)
    L[np.arange(len(rows))[rows < w], rows[rows < w]] = 1.0
    U = np.triu(got[:w])
    lu = L @ U
    bound = 4 * w * 2.0 ** -24 * (np.abs(L) @ np.abs(U)) + 1e-30
    assert np.all(np.abs(P.astype(np.float64)[perm[rows]] - lu) <= bound)


@pytest.mark.parametrize("n,nb,pad", [(1000, 64, 37), (2100, 256, 5), (700, 100, 64)])
def test_padded_leading_dimension_with_nan(lp, n, nb, pad):
    """lda > n and ldb > nrhs, padding filled with NaN: factors, solution and
    residual match the unpadded run and the oracle, and the padding is neither
    read into a result nor overwritten."""
    import torch
    nrhs = 3
    A = inputs.matrix(50 + n, n)
    B = inputs.rhs(50 + n, n, nrhs)
    Ap = np.full((n, n + pad), np.nan)
    Ap[:, :n] = A
    Bp = np.full((n, nrhs + 2), np.nan)
    Bp[:, :nrhs] = B
    tAp, tBp = cuda(Ap), cuda(Bp)
    tA0, tB0 = cuda(Ap), cuda(Bp)
    tA, tX = tAp[:, :n], tBp[:, :nrhs]
    ipiv, info = lp.lu_factor(tA, nb, "fp64")
    st = lp.lu_solve(tA, ipiv, info, tX)
    out = host(lp.residual_check(tA0[:, :n], tX, tB0[:, :nrhs]))
    assert int(host(info)[0]) == 0 and int(host(st)[0]) == 0
    got_A, got_B = host(tAp), host(tBp)
    assert np.all(np.isnan(got_A[:, n:])) and np.all(np.isnan(got_B[:, nrhs:]))
    # the unpadded run
    tA2, tX2 = cuda(A), cuda(B)
    ipiv2, info2 = lp.lu_factor(tA2, nb, "fp64")
    lp.lu_solve(tA2, ipiv2, info2, tX2)
    assert np.array_equal(host(ipiv)[:n], host(ipiv2)[:n])
    lu2 = host(tA2)
    assert np.max(np.abs(got_A[:, :n] - lu2)) <= 1e-12 * np.max(np.abs(lu2))
    # the oracle
    lu_o, piv_o, _ = oracle.getrf(A)
    x_o = oracle.getrs(lu_o, piv_o, B)
    assert np.array_equal(host(ipiv)[:n], piv_o)
    x = got_B[:, :nrhs]
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    ro = oracle.residual(A, x, B)
    assert np.all(np.isfinite(out)) and np.all(out[:, 0] < 16)
    assert np.allclose(out[:, 2:], ro[:, 2:], rtol=1e-13, atol=0)
    del torch
