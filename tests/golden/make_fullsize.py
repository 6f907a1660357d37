"""Writes the oracle's solution of a full-size benchmark system.

For one (n, seed) of the synthetic LINPACK workload (A, b uniform on
[-0.5, 0.5), stream 0 and 1 of the seeded generator; paper, section "High
Performance Linpack": A = L U, L y = b, U x = y, scaled residual) this script
runs the binary64 oracle (unblocked elimination with partial pivoting, then
the triangular solves) and stores what the full-size GPU tests compare with:

  fullsize_n<N>_seed<S>.npz   x (float64, n) and ipiv (int32, n)
  fullsize_n<N>_seed<S>.json  scalars: info, the scaled residual and its
                              norms, a Hager-Higham estimate of kappa_inf(A)
                              from the oracle's factors, the relative
                              difference between the oracle's x and a third
                              binary64 solver's (host LAPACK getrf/getrs via
                              scipy: the "noise floor" of x-parity), SHA-256
                              digests of x and ipiv, and the oracle's time.

Every stored value comes from ``oracle/`` (the LAPACK solve only sets the
noise floor).  Memory: one n x n binary64 matrix at a time (8 GiB at
n = 32768).  Run from the repository root, e.g.
    python tests/golden/make_fullsize.py --n 32768 --seed 2202
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402
from oracle import cond  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
GEN_VERSION = "splitmix64-counter-v1"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def log(msg):
    print(f"[make_fullsize] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--seed", type=int, default=2202)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=512)
    args = ap.parse_args()
    n, seed = args.n, args.seed
    if args.threads:
        oracle.set_threads(args.threads)
    threads = oracle.max_threads()
    base = os.path.join(HERE, f"fullsize_n{n}_seed{seed}")

    log(f"n={n} seed={seed} threads={threads}: generating A")
    a = inputs.matrix(seed, n)
    b = inputs.rhs(seed, n, 1)
    log("factoring (oracle, unblocked GEPP)")
    t0 = time.time()
    lu, ipiv, info = oracle.getrf(a, overwrite=True)
    t_factor = time.time() - t0
    log(f"factor done in {t_factor:.1f} s, info={info}")
    if info != 0:
        raise SystemExit(f"singular: info={info}")
    t0 = time.time()
    x = oracle.getrs(lu, ipiv, b)
    t_solve = time.time() - t0
    log(f"solve done in {t_solve:.1f} s")

    # residual on the original A, regenerated row block by row block
    anorm = 0.0
    rnorm = 0.0
    for r0 in range(0, n, args.chunk):
        r1 = min(n, r0 + args.chunk)
        rows = inputs.matrix_rows(seed, n, np.arange(r0, r1))
        r, _ = oracle.row_residuals(rows, x, b[r0:r1])
        rnorm = max(rnorm, float(np.abs(r).max()))
        anorm = max(anorm, float(np.abs(rows).sum(axis=1).max()))
    xnorm = float(np.abs(x).max())
    bnorm = float(np.abs(b).max())
    s = rnorm / (oracle.EPS * (anorm * xnorm + bnorm) * n)
    log(f"scaled residual {s:.4e}")

    xv = np.ascontiguousarray(x.reshape(-1))
    # the solution first: what follows must not lose hours of factorization
    np.savez_compressed(base + ".npz", x=xv, ipiv=ipiv.astype(np.int32))
    log(f"wrote {base}.npz")

    t0 = time.time()
    inv_norm = cond.inv_norm_inf_estimate(lu, ipiv)
    kappa = anorm * inv_norm
    log(f"kappa_inf estimate {kappa:.4e} ({time.time() - t0:.1f} s)")
    # lu is a (factored in place): drop both before A is generated again, or
    # two n x n arrays are alive at once (68.7 GB at n = 65536)
    del lu, a

    # third solver: host LAPACK on A^T's column-major view (= A row-major),
    # solved with trans=1 so that it solves A x = b
    import scipy.linalg as sla
    a = inputs.matrix(seed, n)
    t0 = time.time()
    lu_f, piv_f = sla.lu_factor(a.T, overwrite_a=True, check_finite=False)
    x_lapack = sla.lu_solve((lu_f, piv_f), b, trans=1, check_finite=False)
    t_lapack = time.time() - t0
    del lu_f, a
    noise = float(np.abs(x_lapack - x).max() / np.abs(x).max())
    log(f"LAPACK noise floor {noise:.3e} ({t_lapack:.1f} s)")

    meta = {
        "what": "binary64 oracle solution of the synthetic LINPACK system "
                "(A, b uniform[-0.5,0.5) from the seeded generator, unshifted)",
        "n": n, "seed": seed, "nrhs": 1, "generator": GEN_VERSION,
        "info": info,
        "scaled_residual": s, "r_norm_inf": rnorm, "a_norm_inf": anorm,
        "x_norm_inf": xnorm, "b_norm_inf": bnorm,
        "inv_norm_inf_estimate": inv_norm, "kappa_inf_estimate": kappa,
        "lapack_rel_x_diff": noise,
        "x_sha256": hashlib.sha256(xv.tobytes()).hexdigest(),
        "ipiv_sha256": hashlib.sha256(ipiv.astype(np.int32).tobytes()).hexdigest(),
        "oracle_factor_s": t_factor, "oracle_solve_s": t_solve,
        "oracle_threads": threads, "host_cpu": cpu_model(), "host_nproc": os.cpu_count(),
        "lapack_s": t_lapack,
        "written_by": "tests/golden/make_fullsize.py (oracle/ only; scipy for the noise floor)",
    }
    with open(base + ".json", "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    log(f"wrote {base}.npz/.json")


if __name__ == "__main__":
    main()
