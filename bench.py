"""Benchmark of the dense LU solve path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 32768] [--nb 256]

One step is one pass of the whole path over one synthetic system: blocked LU
factorization with partial pivoting (panel, row exchanges, triangular solve,
inner-block update, look-ahead), forward/back substitution and the benchmark's
scaled-residual check.  The K systems are generated on the device and copied
into K separate buffers before the timed region, so every timed step starts
from inputs already resident in HBM.  `value` is K * (2/3 n^3 + 2 n^2) flops
over the wall time of the K steps (LINPACK's operation count).

The line also carries the roofline of the dominant kernel (the FP64 trailing
update, bound by the FP64 matrix-core peak), measured with HIP events around
each of its launches during the timed steps, and the CPU oracle timed on a
bounded sample on this host.  Rank 0 prints one JSON line on stdout; progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LU solve TFLOP/s FP64 vs mixed+IR at scaled residual<16; serve p50/p99 ms"
PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix peak (spec sheet)
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops(n: int, nrhs: int = 1) -> float:
    return 2.0 / 3.0 * n ** 3 + 2.0 * n ** 2 * nrhs


def cpu_baseline(n: int, seed: int) -> dict:
    """The oracle (unblocked GEPP + solves) on this host, on one n x n system."""
    import oracle
    import inputs
    a = inputs.matrix(seed, n)
    b = inputs.rhs(seed, n, 1)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    lu, piv, info = oracle.getrf(a, overwrite=True)
    x = oracle.getrs(lu, piv, b)
    dt = time.perf_counter() - t0
    return {"value": flops(n) / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle", "seconds": dt,
            "sample": f"one FP64 system n={n} (LU with partial pivoting + solve), "
                      f"uniform[-0.5,0.5) seed {seed}; same operation count formula"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2202)
    ap.add_argument("--no-lookahead", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="run a plain element-wise copy-convert of this many MiB of doubles "
                         "before the timed steps (reference for HBM traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path runs on one GPU's share); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        return 2

    import torch
    import inputs
    import paper_2202_13995_amd as lp

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    n, nb, K, W = args.n, args.nb, args.steps, args.warmup
    free, total = torch.cuda.mem_get_info()
    need = (K + 2) * 8 * n * n
    if need > 0.9 * free:
        K = max(1, int(0.9 * free // (8 * n * n)) - 2)
        log(f"[bench] memory allows {K} timed copies")
    log(f"[bench] n={n} nb={nb} steps={K} warmup={W} free={free / 2**30:.1f} GiB")

    A0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    inputs.fill_matrix_(A0, args.seed)
    B0 = torch.empty((n, args.nrhs), dtype=torch.float64, device=dev)
    inputs.fill_rhs_(B0, args.seed)
    work = lp.workspace(n, nb, "fp64", dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    look = not args.no_lookahead

    calib = None
    if args.calib_mib > 0:
        rows = max(1, args.calib_mib * 2**20 // (8 * n))
        src = A0[:rows]
        dst = torch.empty((rows, n), dtype=torch.float32, device=dev)
        lp.convert(src, dst)
        torch.cuda.synchronize()
        calib = {"kernel": "convert_kernel<double,float>", "read_bytes": 8 * rows * n,
                 "write_bytes": 4 * rows * n}
        del dst

    # warm-up on a scratch copy
    scratch = torch.empty_like(A0)
    for w in range(W):
        scratch.copy_(A0)
        X = B0.clone()
        lp.lu_factor(scratch, nb, "fp64", work=work, ipiv=ipiv, info=info, lookahead=look)
        lp.lu_solve(scratch, ipiv, info, X)
        lp.residual_check(A0, X, B0)
        torch.cuda.synchronize()
        log(f"[bench] warm-up {w + 1}/{W} done")
    del scratch

    As = [A0.clone() for _ in range(K)]
    Xs = [B0.clone() for _ in range(K)]
    outs = [torch.empty((args.nrhs, 5), dtype=torch.float64, device=dev) for _ in range(K)]
    infos = [torch.empty(1, dtype=torch.int32, device=dev) for _ in range(K)]
    profs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        _, _, prof = lp.lu_factor(As[i], nb, "fp64", work=work, ipiv=ipiv, info=infos[i],
                                  lookahead=look, profile=True)
        lp.lu_solve(As[i], ipiv, infos[i], Xs[i])
        lp.residual_check(A0, Xs[i], B0, out=outs[i])
        profs.append(prof)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    log(f"[bench] timed {K} steps in {elapsed:.3f} s")

    res = torch.stack(outs).cpu().numpy()
    s_max = float(res[:, :, 0].max())
    info_ok = all(int(t.item()) == 0 for t in infos)
    if not (info_ok and s_max < 16.0):
        log(f"[bench] RESIDUAL CHECK FAILED: max scaled residual {s_max}, info ok {info_ok}")

    total_flops = K * flops(n, args.nrhs)
    value = total_flops / elapsed / 1e12
    gemm_ms = sum(p["gemm_ms"] for p in profs)
    gemm_flops = sum(p["gemm_flops"] for p in profs)
    gemm_launches = sum(p["gemm_launches"] for p in profs)
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    phases = {k: sum(p[k] for p in profs) / K for k in
              ("gemm_ms", "panel_ms", "swap_ms", "trsm_ms")}
    phases["gemm_launches_per_step"] = gemm_launches / K
    phases["gemm_avg_launch_us"] = 1e3 * gemm_ms / max(gemm_launches, 1)
    phases["gemm_avg_launch_gflop"] = gemm_flops / max(gemm_launches, 1) / 1e9
    swap_bytes = sum(p["swap_bytes"] for p in profs)
    swap_ms = sum(p["swap_ms"] for p in profs)
    phases["swap_GBps"] = swap_bytes / (swap_ms * 1e-3) / 1e9 if swap_ms > 0 else 0.0

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 blocked LU with partial pivoting + solve + residual "
                               f"check, n={n}, nb={nb}, nrhs={args.nrhs}, A and b "
                               f"uniform[-0.5,0.5) seed {args.seed}",
                   "n": n, "nb": nb, "nrhs": args.nrhs, "lookahead": look},
        "frac_fp64_peak": value / PEAK_FP64_TFLOPS,
        "scaled_residual_max": s_max,
        "residual_pass": bool(info_ok and s_max < 16.0),
        "roofline": {"kernel": "dgemm_trailing_update", "bound": "mfma",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None},
        "phases_ms_per_step": phases,
    }
    if calib is not None:
        line["calibration"] = calib
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle sample n={args.cpu_n} ...")
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, args.seed)
        log(f"[bench] CPU oracle took {line['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
