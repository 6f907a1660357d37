"""Single workloads of the solver, for profilers.

    python -m paper_2202_13995_amd.workloads fp64   [--n 65536 --nb 512 --reps 1]
    python -m paper_2202_13995_amd.workloads nopiv  [--n 65536 --nb 512 --shift]
    python -m paper_2202_13995_amd.workloads mixed  [--n 65536 --nb 512 --prec bf16 --shift]
    python -m paper_2202_13995_amd.workloads solve  [--n 65536 --prec fp32]
    python -m paper_2202_13995_amd.workloads ptrans [--n 32768 --prec fp64]
    python -m paper_2202_13995_amd.workloads copy   [--mib 1024]

Each runs the named path on seeded synthetic inputs (generated on the device
before anything is timed) `reps` times and prints one line per repetition, so
that a profiler's per-kernel summary covers exactly that path:
  fp64   LU with partial pivoting + solve + residual check (look-ahead on);
  nopiv  the same without row exchanges (lu_factor_nopiv);
  mixed  the low-precision factorization + binary64 refinement (lu_solve_ir);
  solve  the triangular solves alone, on factors of the given storage;
  ptrans C = B + A^T;
  copy   a plain element-wise binary64 -> binary32 conversion of a known
         number of bytes (the reference for scaling traffic counters).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["fp64", "nopiv", "mixed", "solve", "ptrans", "copy"])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--prec", default=None)
    ap.add_argument("--shift", action="store_true", help="add n to the diagonal")
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2202)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--gmres", type=int, default=1,
                    help="mixed: 0 classical refinement only, 1 GMRES when it stalls, 2 GMRES")
    args = ap.parse_args(argv)

    import torch

    import inputs
    import paper_2202_13995_amd as lp

    dev = torch.device("cuda:0")
    n, nb = args.n, args.nb
    shift = float(n) if args.shift else 0.0

    def say(msg):
        print(f"[workload {args.what}] {msg}", flush=True)

    if args.what == "copy":
        rows = max(1, args.mib * 2**20 // (8 * 8192))
        src = torch.empty((rows, 8192), dtype=torch.float64, device=dev)
        inputs.fill_matrix_(src, args.seed, logical_cols=8192)
        dst = torch.empty((rows, 8192), dtype=torch.float32, device=dev)
        for r in range(args.reps):
            lp.convert(src, dst)
            torch.cuda.synchronize()
            say(f"rep {r}: read {8 * rows * 8192} B, wrote {4 * rows * 8192} B")
        return 0

    if args.what == "ptrans":
        dt = torch.float32 if args.prec == "fp32" else torch.float64
        A = torch.empty((n, n), dtype=dt, device=dev)
        inputs.fill_matrix_(A, args.seed)
        B = torch.empty((n, n), dtype=dt, device=dev)
        inputs.fill_matrix_(B, args.seed + 1)
        C = torch.empty_like(B)
        for r in range(args.reps):
            lp.ptrans(A, B, C)
            torch.cuda.synchronize()
            say(f"rep {r} done")
        return 0

    A0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    inputs.fill_matrix_(A0, args.seed, shift=shift)
    B0 = torch.empty((n, 1), dtype=torch.float64, device=dev)
    inputs.fill_rhs_(B0, args.seed)
    torch.cuda.synchronize()

    if args.what == "mixed":
        prec = args.prec or "bf16"
        X = torch.empty_like(B0)
        nbytes = lp.lib.lu_solve_ir_workspace_bytes(n, nb, lp.PREC[prec], 1)
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for r in range(args.reps):
            t0 = time.perf_counter()
            _, rep = lp.solve_ir(A0, B0, nb, prec, X=X, work=work, gmres=args.gmres)
            d = rep.as_dict()
            say(f"rep {r}: {1e3 * (time.perf_counter() - t0):.1f} ms, {d['iterations']} "
                f"corrections ({d['gmres_corrections']} GMRES, {d['gmres_steps']} steps), "
                f"fell back {d['fell_back']}, history {d['history']}, phases "
                f"factor {d['t_factor_ms']:.0f} refine {d['t_refine_ms']:.0f} "
                f"fallback {d['t_fallback_ms']:.0f} ms")
        return 0

    if args.what == "solve":
        prec = args.prec or "fp64"
        dt = torch.float64 if prec == "fp64" else torch.float32
        F = A0.to(dt)
        del A0
        ipiv, info = lp.lu_factor_nopiv(F, nb, prec) if args.shift else lp.lu_factor(F, nb, prec)
        X = B0.to(dt)
        torch.cuda.synchronize()
        for r in range(args.reps):
            X.copy_(B0)
            t0 = time.perf_counter()
            lp.lu_solve(F, ipiv, info, X)
            torch.cuda.synchronize()
            say(f"rep {r}: {1e3 * (time.perf_counter() - t0):.2f} ms")
        return 0

    A = torch.empty_like(A0)
    X = torch.empty_like(B0)
    work = lp.workspace(n, nb, "fp64", dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    for r in range(args.reps):
        A.copy_(A0)
        X.copy_(B0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.what == "nopiv":
            lp.lu_factor_nopiv(A, nb, "fp64", work=work, ipiv=ipiv, info=info)
        else:
            lp.lu_factor(A, nb, "fp64", work=work, ipiv=ipiv, info=info)
        lp.lu_solve(A, ipiv, info, X)
        out = lp.residual_check(A0, X, B0)
        torch.cuda.synchronize()
        say(f"rep {r}: {1e3 * (time.perf_counter() - t0):.1f} ms, scaled residual "
            f"{float(out[0, 0].item()):.3e}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
