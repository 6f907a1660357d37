"""GPU parity for the PTRANS kernel, C = B + A^T (paper, section "Parallel
Matrix Transposition").  One rounded addition per element: the GPU result
must equal the oracle's bit for bit, in binary64 and binary32, for ragged
sizes (not multiples of the 64 x 64 tile), padded leading dimensions (the
padding must stay untouched), in place (C = B), and at full size on sampled
rows and columns."""
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


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 1000, 4097])
def test_ptrans_bit_exact(lp, n, dtype):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, (n, n)).astype(dtype)
    b = rng.uniform(-1, 1, (n, n)).astype(dtype)
    c = host(lp.ptrans(cuda(a), cuda(b)))
    assert np.array_equal(c, oracle.ptrans(a, b))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_ptrans_padded_and_in_place(lp, dtype):
    import torch
    n, pad = 777, 19
    rng = np.random.default_rng(5)
    a = rng.uniform(-1, 1, (n, n)).astype(dtype)
    b = rng.uniform(-1, 1, (n, n)).astype(dtype)
    ap = np.full((n, n + pad), np.nan, dtype=dtype)
    ap[:, :n] = a
    bp = np.full((n, n + pad), np.nan, dtype=dtype)
    bp[:, :n] = b
    tAp, tBp = cuda(ap), cuda(bp)
    lp.ptrans(tAp[:, :n], tBp[:, :n], C=tBp[:, :n])  # in place into B
    got = host(tBp)
    assert np.array_equal(got[:, :n], oracle.ptrans(a, b))
    assert np.all(np.isnan(got[:, n:]))
    assert np.array_equal(host(tAp)[:, :n], a)
    del torch


def test_ptrans_fullsize_sampled(lp):
    """n = 32768 binary64 (the LINPACK matrix size of this build): sampled rows
    and columns of C against the definition on host-generated rows of A, B."""
    import torch
    n, seed = 32768, 2202
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    inputs.fill_matrix_(A, seed)
    B = torch.empty((n, n), dtype=torch.float64, device="cuda")
    inputs.fill_matrix_(B, seed + 1)
    C = lp.ptrans(A, B)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([[0, 63, 64, n - 1], rng.integers(0, n, 12)]))
    c_rows = C.index_select(0, torch.from_numpy(rows).cuda()).cpu().numpy()
    b_rows = inputs.matrix_rows(seed + 1, n, rows)
    # column i of A (= row i of A^T) from host rows of A: sample the columns too
    cols = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 12)]))
    a_cols_rows = inputs.matrix_rows(seed, n, cols)           # rows `cols` of A
    for t, i in enumerate(rows):
        ref = b_rows[t, cols] + a_cols_rows[:, i]              # c_ij = b_ij + a_ji
        assert np.array_equal(c_rows[t, cols], ref)
    # A untouched: its sampled rows equal the generator
    a_rows = A.index_select(0, torch.from_numpy(cols).cuda()).cpu().numpy()
    assert np.array_equal(a_rows, a_cols_rows)
