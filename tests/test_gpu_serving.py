"""GPU tests of the continuous-batching server.

Every request's result is checked against the CPU oracle (x within 1e-10,
scaled residual < 16), the same request gives bitwise the same x alone and in
a mix, admission respects the memory pool, and failures are reported.
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


def make(n, nrhs, seed, shift=0.0):
    import torch
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    inputs.fill_matrix_(A, seed, shift=shift)
    B = torch.empty((n, nrhs), dtype=torch.float64, device="cuda")
    inputs.fill_rhs_(B, seed)
    X = torch.full((n, nrhs), float("nan"), dtype=torch.float64, device="cuda")
    return A, B, X


MIX = [(64, 1, "fp64"), (100, 3, "fp32"), (257, 8, "fp64"), (511, 2, "bf16"), (700, 1, "fp64"),
       (1500, 4, "fp32"), (96, 5, "fp64"), (2048, 2, "fp64"), (130, 1, "fp16"), (33, 7, "fp64")]


U64 = 2.0 ** -53


def check_against_oracle(A, B, X, seed, n, nrhs, prec="fp64"):
    """Scaled residual < 16 by the oracle's own check, and the forward error.

    Binary64 requests agree with the oracle's solution to 1e-10 (rounding-order
    differences only).  Low-precision requests stop refining once the scaled
    residual s is below 16, which bounds |x - x*| / |x*| by about
    kappa_inf(A) * 2 * s * n * u; with the oracle's own error of kappa * n * u on
    top, the bound checked is 48 * kappa_inf(A) * n * u."""
    a = inputs.matrix(seed, n)
    b = inputs.rhs(seed, n, nrhs)
    x = X.cpu().numpy()
    x_o = oracle.solve(a, b)
    err = np.max(np.abs(x - x_o)) / np.max(np.abs(x_o))
    if prec == "fp64":
        tol = 1e-10
    else:
        kappa = np.linalg.norm(a, np.inf) * np.linalg.norm(np.linalg.inv(a), np.inf)
        tol = 48 * kappa * n * U64
    assert err <= tol, (n, nrhs, prec, err, tol)
    assert np.all(oracle.residual(a, x, b)[:, 0] < 16), (n, nrhs, prec)


def test_mixed_stream_matches_oracle(lp):
    import torch
    with lp.Server(memory_bytes=1 << 30, small_n_max=512, max_batch=64, batch_slots=3,
                   large_slots=2) as sv:
        reqs = {}
        for i, (n, nrhs, prec) in enumerate(MIX):
            A, B, X = make(n, nrhs, 1000 + i)
            t = sv.submit(A, B, X, prec=prec, nb=64)
            reqs[t] = (A, B, X, 1000 + i, n, nrhs, prec)
        results = sv.drain()
    torch.cuda.synchronize()
    assert sorted(r["ticket"] for r in results) == sorted(reqs)
    for r in results:
        A, B, X, seed, n, nrhs, prec = reqs[r["ticket"]]
        assert r["status"] == 0 and r["info"] == 0, r
        assert r["scaled_residual"] < 16, r
        assert r["batched"] == (1 if n <= 512 else 0)
        # the request's own device time is part of its latency
        assert 0.0 < r["device_ms"] <= r["latency_ms"] + 1e-3, r
        check_against_oracle(A, B, X, seed, n, nrhs, prec)


def test_same_result_alone_and_in_a_mix(lp):
    import torch
    probe = [(300, 2, "fp64", 7), (400, 1, "fp32", 8), (1200, 3, "fp64", 9), (900, 2, "bf16", 10)]
    alone = {}
    for n, nrhs, prec, seed in probe:
        with lp.Server(memory_bytes=1 << 30, small_n_max=512) as sv:
            A, B, X = make(n, nrhs, seed)
            sv.submit(A, B, X, prec=prec, nb=64)
            sv.drain()
            torch.cuda.synchronize()
            alone[seed] = X.cpu().numpy().copy()
    with lp.Server(memory_bytes=1 << 30, small_n_max=512, max_batch=16, batch_slots=4,
                   large_slots=3) as sv:
        mine = {}
        k = 0
        for n, nrhs, prec, seed in probe:
            # interleave with other traffic
            for j in range(3):
                A2, B2, X2 = make(64 + 97 * j + 13 * k, 1 + j, 5000 + 10 * k + j)
                sv.submit(A2, B2, X2, prec="fp64" if j % 2 else "fp32", nb=64)
            A, B, X = make(n, nrhs, seed)
            sv.submit(A, B, X, prec=prec, nb=64)
            mine[seed] = X
            k += 1
            sv.poll()
        sv.drain()
    torch.cuda.synchronize()
    for seed, X in mine.items():
        assert np.array_equal(X.cpu().numpy(), alone[seed]), seed


def test_admission_by_footprint(lp):
    import torch
    A, B, X = make(400, 1, 3)
    with lp.Server(memory_bytes=8 << 20, small_n_max=512, max_batch=8) as sv:
        foot = sv.footprint(A, B, X, prec="fp64")
        assert 0 < foot < (8 << 20)
        # more requests than the pool holds at once: they queue and all finish
        items = [make(400, 1, 20 + i) for i in range(12)]
        for a, b, x in items:
            sv.submit(a, b, x, prec="fp64")
        seen_queue = False
        out = []
        while len(out) < len(items):
            q, r, used = sv.pending()
            assert used <= (8 << 20)
            seen_queue |= q > 0
            out += sv.poll()
        assert seen_queue
        assert all(r["status"] == 0 for r in out)
        # a request that can never fit is rejected at submission
        big = make(2000, 1, 4)
        with pytest.raises(lp.LPError) as e:
            sv.submit(*big, prec="fp64")
        assert e.value.code == lp.LP_ENOSPC
    torch.cuda.synchronize()
    for i, (a, b, x) in enumerate(items):
        check_against_oracle(a, b, x, 20 + i, 400, 1)


def test_singular_request_reports_failure(lp):
    import torch
    with lp.Server(memory_bytes=1 << 28, small_n_max=512) as sv:
        A, B, X = make(200, 1, 6)
        A[:, 7] = 0.0
        A2, B2, X2 = make(800, 1, 6)
        A2[:, 9] = 0.0
        sv.submit(A, B, X, prec="fp64")
        sv.submit(A2, B2, X2, prec="fp64", nb=64)
        res = sorted(sv.drain(), key=lambda r: r["ticket"])
    assert res[0]["status"] == 1 and res[0]["info"] == 8
    assert res[1]["status"] == 1 and res[1]["info"] == 10


def test_shifted_mixed_requests_refine(lp):
    import torch
    with lp.Server(memory_bytes=1 << 30, small_n_max=512) as sv:
        items = []
        for i, n in enumerate((128, 1024)):
            A, B, X = make(n, 2, 70 + i, shift=float(n))
            sv.submit(A, B, X, prec="bf16", nb=128)
            items.append((A, B, X, n))
        res = sv.drain()
    for r in res:
        assert r["status"] == 0 and r["fell_back"] == 0 and r["scaled_residual"] < 16, r
