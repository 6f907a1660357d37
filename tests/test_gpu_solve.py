"""GPU parity for the two triangular-solve paths (paper, section "High
Performance Linpack": L y = b, then U x = y, after the row interchanges).

lu_solve runs one launch pair per 128-row block; lu_solve_ex runs each
triangle as one persistent launch whose workgroups pull already solved blocks
through tagged words.  Both are compared with the oracle's substitution on
the same factors (the oracle's own factorization, uploaded), so only the
solves are under test: x within a bound derived from the arithmetic, ragged
sizes, several passes of right-hand sides, binary32 storage, and a singular
factorization that must leave B untouched."""
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


@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (2, 3), (127, 1), (128, 2), (129, 8), (1031, 11),
                                    (2048, 1), (3001, 4), (5000, 17)])
def test_solve_against_oracle_substitution(lp, n, nrhs, persistent):
    import torch
    a = inputs.matrix(400 + n, n)
    b = inputs.rhs(400 + n, n, nrhs)
    lu_o, piv_o, info_o = oracle.getrf(a)
    x_o = oracle.getrs(lu_o, piv_o, b)
    tLU = cuda(lu_o)
    ipiv = cuda(piv_o.astype(np.int32))
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    X = cuda(b)
    st = lp.lu_solve(tLU, ipiv, info, X, persistent=persistent)
    assert int(host(st)[0]) == 0
    x = host(X)
    # the same factors, another summation order: forward error ~ cond * n * eps
    assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10
    assert np.all(oracle.residual(a, x, b)[:, 0] < 16)
    assert np.array_equal(host(tLU), lu_o)  # the factors are read only


@pytest.mark.parametrize("n,nrhs", [(1000, 3), (4099, 9)])
def test_solve_binary32_storage(lp, n, nrhs):
    import torch
    a32 = inputs.matrix(7 + n, n, shift=float(n)).astype(np.float32)
    b32 = inputs.rhs(7 + n, n, nrhs).astype(np.float32)
    lu_o, piv_o, _ = oracle.getrf(a32.astype(np.float64))
    lu32 = lu_o.astype(np.float32)
    # reference: the substitution in binary64 on the same binary32 factors
    x_ref = oracle.getrs(lu32.astype(np.float64), piv_o, b32.astype(np.float64))
    for persistent in (True, False):
        X = cuda(b32)
        lp.lu_solve(cuda(lu32), cuda(piv_o.astype(np.int32)),
                    torch.zeros(1, dtype=torch.int32, device="cuda"), X, persistent=persistent)
        x = host(X).astype(np.float64)
        assert np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)) <= 64 * n * 2.0 ** -24


def test_solve_refuses_singular_factors(lp):
    import torch
    n = 300
    a = inputs.matrix(3, n)
    lu_o, piv_o, _ = oracle.getrf(a)
    b = inputs.rhs(3, n, 2)
    for persistent in (True, False):
        X = cuda(b)
        info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        st = lp.lu_solve(cuda(lu_o), cuda(piv_o.astype(np.int32)), info, X,
                         persistent=persistent)
        assert int(host(st)[0]) == 1
        assert np.array_equal(host(X), b)


def test_solve_workspace_checks(lp):
    L = lp.lib
    assert L.lu_solve_workspace_bytes(1000, 0, 1) > L.lu_solve_workspace_bytes(1000, 1, 1)
    assert L.lu_solve_workspace_bytes(-1, 0, 1) == 0
    assert L.lu_solve_workspace_bytes(10, 2, 1) == 0
    import ctypes
    p = ctypes.c_void_p(256)
    assert L.lu_solve_ex(10, 0, p, 10, p, p, p, 1, 1, None, p, 0, None) == lp.LP_ENOSPC
