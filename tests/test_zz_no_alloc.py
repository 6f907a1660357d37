"""The allocation-free factorization entry point (lu_factor_noalloc).

It runs the same partial-pivoting factorization as lu_factor, strictly in
order on the caller's stream, with its workspace in a file-scope device array
instead of a caller buffer.  Called through the C ABI twice in a row, the
second time on a smaller system (so the array holds the first call's leftovers),
and compared with lu_factor_ex without look-ahead (the same kernels and launch
shapes: pivots and factors bit for bit), with the default lu_factor (factors
within 1e-12), and with the oracle (pivots bit-exact, x within 1e-10).
"""
import ctypes

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


def noalloc(lp, A, nb, prec):
    import torch
    n = A.shape[0]
    ipiv = torch.full((n,), -1, dtype=torch.int32, device=A.device)
    info = torch.full((1,), -5, dtype=torch.int32, device=A.device)
    rc = lp.lib.lu_factor_noalloc(n, nb, prec, A.data_ptr(), A.stride(0), ipiv.data_ptr(),
                                  info.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0, lp.strerror(rc)
    return ipiv, info


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_lu_factor_twice(lp, prec):
    import torch
    dt = torch.float64 if prec == 0 else torch.float32
    name = "fp64" if prec == 0 else "fp32"
    for n, nb, seed in ((3000, 128, 71), (1000, 64, 72)):
        print(f"lu_factor_noalloc n={n} nb={nb} prec={name}", flush=True)
        a = inputs.matrix(seed, n)
        A1 = torch.from_numpy(a).to(device="cuda", dtype=dt)
        A2 = A1.clone()
        A3 = A1.clone()
        ipiv1, info1 = noalloc(lp, A1, nb, prec)
        ipiv2, info2 = lp.lu_factor(A2, nb, name, lookahead=False)
        ipiv3, info3 = lp.lu_factor(A3, nb, name)
        torch.cuda.synchronize()
        assert int(info1.item()) == int(info2.item()) == 0
        assert torch.equal(ipiv1, ipiv2[:n]) and torch.equal(A1, A2)
        if prec == 0:
            # the default (look-ahead) schedule: same pivots, factors to rounding
            assert torch.equal(ipiv1, ipiv3[:n])
            d = float((A1 - A3).abs().max()) / float(A3.abs().max())
            assert d <= 1e-12
            lu_o, piv_o, _ = oracle.getrf(a)
            assert np.array_equal(ipiv1.cpu().numpy(), piv_o)
            b = inputs.rhs(seed, n, 1)
            X = torch.from_numpy(b).cuda()
            lp.lu_solve(A1, ipiv1, info1, X)
            x_o = oracle.getrs(lu_o, piv_o, b)
            x = X.cpu().numpy()
            assert np.max(np.abs(x - x_o)) / np.max(np.abs(x_o)) <= 1e-10


def test_noalloc_limits(lp):
    L = lp.lib
    assert L.lu_factor_noalloc_max_bytes() == 8 << 20
    assert L.lu_workspace_bytes(131072, 1024, 0) <= L.lu_factor_noalloc_max_bytes()
    # bfloat16 storage needs packed operands: refused before touching the device
    assert L.lu_factor_noalloc(100, 32, 2, ctypes.c_void_p(16), 100, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), None) == lp.LP_ENOTSUP
    assert L.lu_factor_noalloc(-1, 32, 0, None, 1, None, None, None) == -1
