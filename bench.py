"""Benchmark of the dense LU solve path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 65536] [--nb 512]

One step is one pass of the whole path over one synthetic system: blocked LU
factorization with partial pivoting (panel, row exchanges, triangular solve,
inner-block update, look-ahead), forward/back substitution and the benchmark's
scaled-residual check.  The default workload is the largest single-GPU
configuration: n = 65536, nb = 512, A and b uniform[-0.5, 0.5) from seed 2202,
unshifted.  The system is generated once on the device; before every step
(warm-up and timed) the working matrix and right-hand side are restored from
that copy outside the timed interval, so every timed step starts from inputs
already resident in HBM.  Each step is bracketed by device synchronizations
and timed on the host clock; `value` is K * (2/3 n^3 + 2 n^2) flops over the
sum of the K step times (LINPACK's operation count), and the best, median and
mean step times are reported beside it.

The line also carries the roofline of the dominant kernel (the FP64 trailing
update, bound by the FP64 matrix-core peak), measured with HIP events around
each of its launches during the timed steps, its HBM traffic per launch from
the committed rocprofv3 counter summary (null if the kernel source changed
since), and the CPU oracle timed on a bounded sample on this host.

More objects ride on the same line:
  * `x_parity`: the binary64 path at n = 32768 against the oracle's stored
    solution of that system (forward error next to the host-LAPACK noise
    floor, pivot agreement), when the stored solution is present;
  * `mixed_ir` (n = 65536 solved through the bfloat16 factorization plus
    binary64 refinement on A + n I, with the binary64 path timed on that same
    system the same number of times for the speedup);
  * `mixed_ir_unshifted` (the same route on the unshifted headline system:
    refinement history -- classical, then GMRES corrections -- fallback, and
    the time with and without it), and `mixed_ir_unshifted_fp32` (binary32
    update operands on that system, where refinement converges);
  * `ptrans` (the paper's matrix transposition kernel C = B + A^T at
    n = 32768: achieved GB/s against the HBM peak, and the paper's n^2
    additions per second);
  * `serving` (the continuous-batching server: saturation measured with a
    burst, then open-loop Poisson streams at 25/50/80% of it, 2000 requests
    each: p50/p99 latency overall and per request class, aggregate TFLOP/s).
One process, one GPU; prints one JSON line on stdout, progress on stderr.
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


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    out = {"value": flops(n) / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
           "kind": "oracle", "seconds": dt,
           "host_cpu": host_cpu_model(), "host_nproc": os.cpu_count(),
           "sample": f"one FP64 system n={n} (LU with partial pivoting + solve), "
                     f"uniform[-0.5,0.5) seed {seed}; same operation count formula"}
    # the small configuration (n = 1024) on one thread and on all of them
    small = {}
    for t in (1, threads):
        oracle.set_threads(t)
        a = inputs.matrix(seed, 1024)
        b = inputs.rhs(seed, 1024, 1)
        t0 = time.perf_counter()
        lu, piv, info = oracle.getrf(a, overwrite=True)
        oracle.getrs(lu, piv, b)
        small[f"threads_{t}_s"] = time.perf_counter() - t0
    oracle.set_threads(threads)
    out["n1024"] = small
    return out


def stats_ms(times_s) -> dict:
    import statistics
    ms = [1e3 * t for t in times_s]
    return {"best_ms": min(ms), "median_ms": statistics.median(ms),
            "mean_ms": sum(ms) / len(ms), "reps": len(ms)}


def load_golden(n: int, seed: int):
    """The oracle's stored solution of the (n, seed) system, or None."""
    import numpy as np
    base = os.path.join(ROOT, "tests", "golden", f"fullsize_n{n}_seed{seed}")
    if not os.path.exists(base + ".npz"):
        return None
    with np.load(base + ".npz", allow_pickle=False) as z:
        g = {"x": z["x"], "ipiv": z["ipiv"]}
    with open(base + ".json") as f:
        g.update(json.load(f))
    return g


def forward_error(x, x_ref) -> float:
    """max |x - x_ref| / max |x_ref| (device tensors or host arrays)."""
    import numpy as np

    def host(v):
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
        return np.asarray(v, dtype=np.float64).reshape(-1)
    x, r = host(x), host(x_ref)
    return float(np.max(np.abs(x - r)) / np.max(np.abs(r)))


def bench_x_parity(lp, inputs, torch, dev, n, nb, seed):
    """The binary64 path on the (n, seed) system against the oracle's stored
    solution: forward error, the host-LAPACK noise floor and kappa estimate
    stored with it, pivot agreement, and both scaled residuals."""
    import numpy as np
    g = load_golden(n, seed)
    if g is None:
        return None
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    inputs.fill_matrix_(A, seed)
    B = torch.empty((n, 1), dtype=torch.float64, device=dev)
    inputs.fill_rhs_(B, seed)
    A0 = A.clone()
    X = B.clone()
    ipiv, info = lp.lu_factor(A, nb, "fp64")
    lp.lu_solve(A, ipiv, info, X)
    out = lp.residual_check(A0, X, B).cpu().numpy()
    piv = ipiv.cpu().numpy()[:n]
    rel = forward_error(X, g["x"])
    del A, A0
    torch.cuda.empty_cache()
    return {"n": n, "nb": nb, "seed": seed,
            "forward_error_vs_oracle": rel,
            "noise_floor_lapack_vs_oracle": g["lapack_rel_x_diff"],
            "kappa_inf_estimate": g["kappa_inf_estimate"],
            "pivot_agreement": float(np.mean(piv == g["ipiv"])),
            "scaled_residual": float(out[0, 0]),
            "oracle_scaled_residual": g["scaled_residual"],
            "oracle_factor_s": g["oracle_factor_s"], "oracle_threads": g["oracle_threads"],
            "oracle_host_cpu": g["host_cpu"]}


PEAK_LOWP_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}  # dense MFMA peaks


def traffic_from_profile(kernel_src: str, n: int, nb: int):
    """HBM bytes per launch of the trailing update from the committed rocprofv3
    counter summary, or None when there is none for this workload or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"dgemm_trailing_update_n{n}_nb{nb}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_b):
        return None
    src = open(os.path.join(ROOT, "paper_2202_13995_amd", "csrc", kernel_src), "rb").read()
    if hashlib.sha256(src).hexdigest() != m_sha.group(1):
        return None
    return float(m_b.group(1))


def bench_mixed(lp, inputs, torch, dev, n, nb, prec, shift, seed, R, nrhs, fp64_leg=True,
                x_ref=None, x_ref_label=None, nopiv_leg=False, fp64_nb=None):
    """R timed solves (after one untimed) of one system through the
    low-precision factorization plus binary64 refinement (and the binary64
    fallback when refinement fails).  With fp64_leg the binary64 blocked path
    is timed on that same system the same way, for the speedup (and with
    nopiv_leg the binary64 path without row exchanges too).  The forward
    error is taken against x_ref (the oracle's or the binary64 path's x) and
    the backward error is the scaled residual.  The binary64 legs use block
    fp64_nb (default nb): each path at its own best block size."""
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    inputs.fill_matrix_(A, seed, shift=shift)
    B = torch.empty((n, nrhs), dtype=torch.float64, device=dev)
    inputs.fill_rhs_(B, seed)
    X = torch.empty_like(B)
    nbytes = lp.lib.lu_solve_ir_workspace_bytes(n, nb, lp.PREC[prec], nrhs)
    work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    lp.solve_ir(A, B, nb, prec, X=X, work=work)
    torch.cuda.synchronize()
    reps, times = [], []
    for _ in range(R):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = lp.solve_ir(A, B, nb, prec, X=X, work=work)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        reps.append(rep.as_dict())
    del work
    st = stats_ms(times)
    dt = st["median_ms"] * 1e-3
    last = reps[-1]
    eff = flops(n, nrhs) / dt / 1e12
    res = {
        "workload": f"{prec.upper()} LU (binary32 panels, {prec} update operands, binary32 "
                    f"accumulation) + binary64 refinement to scaled residual < 16, n={n}, "
                    f"nb={nb}, nrhs={nrhs}, A uniform[-0.5,0.5) "
                    + (f"+ {shift:g} I" if shift else "unshifted") + f", seed {seed}",
        "prec": prec, "n": n, "nb": nb, "shift": shift,
        "ms_per_solve": st["median_ms"], "times": st,
        "effective_tflops": eff,
        "effective_over_fp64_peak": eff / PEAK_FP64_TFLOPS,
        "frac_lowp_peak": eff / PEAK_LOWP_TFLOPS[prec],
        # the factorization alone (its 2/3 n^3 flops over its own time)
        "factor_tflops": (2.0 / 3.0) * n ** 3 / (last["t_factor_ms"] * 1e-3) / 1e12,
        "frac_lowp_peak_factor": (2.0 / 3.0) * n ** 3 / (last["t_factor_ms"] * 1e-3) / 1e12
                                 / PEAK_LOWP_TFLOPS[prec],
        "iterations": last["iterations"], "converged": last["converged"],
        "gmres_corrections": last["gmres_corrections"], "gmres_steps": last["gmres_steps"],
        "fell_back": last["fell_back"], "scaled_residual": last["scaled_residual"],
        "backward_error_scaled_residual": last["scaled_residual"],
        "history": last["history"],
        "phase_ms": {k: last[k] for k in ("t_convert_ms", "t_factor_ms", "t_solve0_ms",
                                          "t_refine_ms", "t_fallback_ms", "t_total_ms")},
        "ms_without_fallback": last["t_total_ms"] - last["t_fallback_ms"],
        "residual_pass": bool(last["scaled_residual"] < 16.0),
    }
    if fp64_leg:
        A64 = torch.empty_like(A)
        X64 = torch.empty_like(B)
        nb64 = fp64_nb or nb
        w64 = lp.workspace(n, nb64, "fp64", dev)
        sw64 = torch.empty(lp.lib.lu_solve_workspace_bytes(n, lp.FP64, nrhs), dtype=torch.uint8,
                           device=dev)
        ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        t64 = []
        out = None
        for r in range(R + 1):
            A64.copy_(A)
            X64.copy_(B)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lp.lu_factor(A64, nb64, "fp64", work=w64, ipiv=ipiv, info=info)
            lp.lu_solve(A64, ipiv, info, X64, work=sw64)
            out = lp.residual_check(A, X64, B)
            torch.cuda.synchronize()
            if r > 0:  # the first solve is the untimed warm-up
                t64.append(time.perf_counter() - t0)
        st64 = stats_ms(t64)
        res["fp64_same_system"] = dict(st64, scaled_residual=float(out[:, 0].max().item()),
                                       nb=nb64)
        res["fp64_ms_same_system"] = st64["median_ms"]
        res["speedup_vs_fp64"] = st64["median_ms"] / st["median_ms"]
        res["forward_error_vs_fp64_path"] = forward_error(X, X64)
        if nopiv_leg:
            # the paper's elimination without row exchanges (valid here: A + n I
            # is diagonally dominant) on the same system: the cost of pivoting
            Xp = X64.clone()
            tn = []
            for r in range(R + 1):
                A64.copy_(A)
                X64.copy_(B)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lp.lu_factor_nopiv(A64, nb64, "fp64", work=w64, ipiv=ipiv, info=info)
                lp.lu_solve(A64, ipiv, info, X64, work=sw64)
                out = lp.residual_check(A, X64, B)
                torch.cuda.synchronize()
                if r > 0:
                    tn.append(time.perf_counter() - t0)
            stn = stats_ms(tn)
            res["fp64_nopiv_same_system"] = dict(
                stn, scaled_residual=float(out[:, 0].max().item()),
                tflops=flops(n, nrhs) / (stn["median_ms"] * 1e-3) / 1e12,
                rel_x_diff_vs_pivoted=forward_error(X64, Xp),
                pivoting_cost=st64["median_ms"] / stn["median_ms"])
        del A64, w64
    if x_ref is not None:
        res["forward_error_vs_" + x_ref_label] = forward_error(X, x_ref)
    del A
    torch.cuda.empty_cache()
    return res


def bench_ptrans(lp, inputs, torch, dev, n, seed, reps):
    """The paper's PTRANS kernel, C = B + A^T, timed with HIP events on the
    stream it runs on (bound by HBM: 3 n^2 elements per call); the paper's
    operation count is n^2 additions."""
    out = {"workload": f"PTRANS C = B + A^T, n={n}, A, B uniform[-0.5,0.5) seeds {seed}, "
                       f"{seed + 1}", "n": n}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        A = torch.empty((n, n), dtype=dt, device=dev)
        inputs.fill_matrix_(A, seed)
        B = torch.empty((n, n), dtype=dt, device=dev)
        inputs.fill_matrix_(B, seed + 1)
        C = torch.empty_like(B)
        lp.ptrans(A, B, C)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            lp.ptrans(A, B, C)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        nbytes = 3.0 * n * n * A.element_size()
        out[name] = {"us_per_call": 1e6 * t, "GBps": nbytes / t / 1e9,
                     "frac_hbm_peak": nbytes / t / 1e9 / PEAK_HBM_GBS,
                     "GFLOPs_paper_metric": n * n / t / 1e9, "bytes_per_call": nbytes}
        del A, B, C
        torch.cuda.empty_cache()
    return out


def serving_requests(inputs, torch, dev, nreq, seed, lowp):
    """The request set of the serving measurements: n = round(exp(U(ln 64,
    ln 4096))), 1-8 right-hand sides, half binary64 and half the low-precision
    route, A and B uniform[-0.5,0.5) with seed + 1 + request index, generated
    on the device before any clock starts."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(64), np.log(4096), nreq)).astype(int)
    nrhs = rng.integers(1, 9, nreq)
    precs = np.where(rng.random(nreq) < 0.5, "fp64", lowp)
    reqs = []
    for i in range(nreq):
        n, r = int(ns[i]), int(nrhs[i])
        A = torch.empty((n, n), dtype=torch.float64, device=dev)
        inputs.fill_matrix_(A, seed + 1 + i)
        B = torch.empty((n, r), dtype=torch.float64, device=dev)
        inputs.fill_rhs_(B, seed + 1 + i)
        reqs.append((A, B, torch.empty_like(B), n, r, str(precs[i])))
    torch.cuda.synchronize()
    return reqs


def serve_stream(lp, torch, sv, reqs, arrivals):
    """One open-loop stream: request i is submitted once arrivals[i] (seconds)
    has passed, whatever is still running (no coordinated omission); its
    latency runs from its arrival time to the poll that returns it."""
    import numpy as np

    def nb_for(n):
        return 64 if n <= 1024 else 128

    nreq = len(reqs)
    t_arr, t_done, res = {}, {}, {}
    i = 0
    t0 = time.perf_counter()
    while len(t_done) < nreq:
        now = time.perf_counter() - t0
        while i < nreq and arrivals[i] <= now:
            A, B, X, n, r, pr = reqs[i]
            t = sv.submit(A, B, X, prec=pr, nb=nb_for(n))
            t_arr[t] = (i, arrivals[i])
            i += 1
        got = sv.poll()
        now = time.perf_counter() - t0
        for d in got:
            t_done[d["ticket"]] = now
            res[d["ticket"]] = d
        if not got and i < nreq and arrivals[i] > now + 2e-4:
            time.sleep(1e-4)
    t_end = time.perf_counter() - t0
    lat = np.array([1e3 * (t_done[t] - t_arr[t][1]) for t in t_done])
    classes = {}
    for t in t_done:
        k = t_arr[t][0]
        n_k, pr_k = reqs[k][3], reqs[k][5]
        key = ("batched" if res[t]["batched"] else "blocked") + "/" + pr_k + \
              ("/n<1024" if n_k < 1024 else "/n>=1024")
        classes.setdefault(key, []).append(1e3 * (t_done[t] - t_arr[t][1]))
    dev_ms = {}
    for t in t_done:
        k = t_arr[t][0]
        key = ("batched" if res[t]["batched"] else "blocked") + "/" + reqs[k][5] + \
              ("/n<1024" if reqs[k][3] < 1024 else "/n>=1024")
        dev_ms.setdefault(key, []).append(res[t]["device_ms"])
    # latency = the request's own device time + the time it waited (admission,
    # a free workgroup or slot, the device shared with other requests)
    by_class = {k: {"count": len(v), "p50_ms": float(np.percentile(v, 50)),
                    "p99_ms": float(np.percentile(v, 99)),
                    "device_p50_ms": float(np.percentile(dev_ms[k], 50)),
                    "device_p99_ms": float(np.percentile(dev_ms[k], 99))}
                for k, v in sorted(classes.items())}
    total = sum(flops(q[3], q[4]) for q in reqs)
    span = t_end - float(arrivals[0])
    bad = [d for d in res.values() if d["status"] != 0 or not d["scaled_residual"] < 16.0]
    return {
        "requests": nreq,
        "achieved_rate_per_s": nreq / span,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
        "aggregate_tflops": total / span / 1e12,
        "makespan_s": span,
        "batched_fraction": float(np.mean([d["batched"] for d in res.values()])),
        "by_class": by_class,
        "fell_back": int(sum(d["fell_back"] for d in res.values())),
        "failed": len(bad),
    }


def bench_serving(lp, inputs, torch, dev, nreq, seed, mem_gib, lowp, small_n_max, large_slots,
                  fractions, burst):
    """Continuous-batching server under open-loop Poisson load.  Saturation is
    measured first with a burst (every request submitted at t = 0: requests per
    second = count / makespan); then arrival rates at the given fractions of
    it, each over the same `nreq` requests."""
    import numpy as np
    reqs = serving_requests(inputs, torch, dev, nreq, seed, lowp)
    with lp.Server(memory_bytes=int(mem_gib * 2**30), small_n_max=small_n_max, max_batch=256,
                   large_slots=large_slots) as sv:
        # warm-up: one request of each route, untimed
        for (n, pr) in ((100, "fp64"), (100, lowp), (1500, "fp64"), (1500, lowp)):
            A = torch.empty((n, n), dtype=torch.float64, device=dev)
            inputs.fill_matrix_(A, 1)
            B = torch.empty((n, 1), dtype=torch.float64, device=dev)
            inputs.fill_rhs_(B, 1)
            sv.submit(A, B, torch.empty_like(B), prec=pr, nb=64 if n <= 1024 else 128)
        sv.drain()
        torch.cuda.synchronize()
        nb_ = min(burst, nreq)
        sat = serve_stream(lp, torch, sv, reqs[:nb_], np.zeros(nb_))
        rate_sat = sat["achieved_rate_per_s"]
        log(f"[bench] serving burst of {nb_}: {rate_sat:.1f} requests/s, p50 {sat['p50_ms']:.1f} ms")
        sweep = []
        rng = np.random.default_rng(seed + 7)
        for f in fractions:
            rate = f * rate_sat
            arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
            r = serve_stream(lp, torch, sv, reqs, arrivals)
            r.update({"fraction_of_saturation": f, "offered_rate_per_s": rate})
            sweep.append(r)
            log(f"[bench] serving at {f:.2f} of saturation ({rate:.1f}/s): p50 {r['p50_ms']:.2f} ms, "
                f"p99 {r['p99_ms']:.2f} ms")
    top = sweep[-1] if sweep else sat
    return {
        "workload": f"Poisson streams of {nreq} requests, n log-uniform [64,4096], 1-8 rhs, half "
                    f"fp64 / half {lowp}+binary64 refinement, A uniform[-0.5,0.5), n<={small_n_max} "
                    f"in the persistent batched kernel, {large_slots} blocked-path slots, pool "
                    f"{mem_gib:g} GiB; arrival rates at {fractions} of the burst-measured saturation",
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
        "aggregate_tflops": top["aggregate_tflops"],
        "saturation": dict(sat, burst_requests=nb_),
        "sweep": sweep,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2202)
    ap.add_argument("--no-lookahead", action="store_true")
    ap.add_argument("--panel-cus", type=int, default=0,
                    help="compute units reserved for short panels (0 never, -1 automatic)")
    ap.add_argument("--panel-rows", type=int, default=0,
                    help="panels of at most this many rows use them (0 default)")
    ap.add_argument("--cpu-n", type=int, default=10240)
    ap.add_argument("--mixed-prec", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--mixed-n", type=int, default=65536,
                    help="order of the mixed-precision system (0: --n)")
    ap.add_argument("--mixed-nb", type=int, default=1024,
                    help="block of the shifted mixed solve (0: --nb); bfloat16 / half "
                         "factorizations are fastest with 1024")
    ap.add_argument("--mixed-unshifted-nb", type=int, default=0,
                    help="block of the unshifted mixed solves (0: --nb)")
    ap.add_argument("--mixed-reps", type=int, default=3,
                    help="timed solves per mixed-precision leg (after one untimed)")
    ap.add_argument("--no-mixed-unshifted", action="store_true",
                    help="skip the unshifted mixed-precision record")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--parity-n", type=int, default=32768,
                    help="order of the system compared with the oracle's stored solution")
    ap.add_argument("--parity-nb", type=int, default=256)
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per arrival rate")
    ap.add_argument("--serve-fractions", default="0.25,0.5,0.8",
                    help="arrival rates as fractions of the measured saturation")
    ap.add_argument("--serve-burst", type=int, default=1000,
                    help="requests of the burst that measures saturation")
    ap.add_argument("--serve-gib", type=float, default=16.0)
    ap.add_argument("--serve-lowp", default="fp32", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--serve-small-n", type=int, default=128,
                    help="requests up to this n run in the persistent batched kernel")
    ap.add_argument("--serve-large-slots", type=int, default=4)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ptrans-n", type=int, default=32768)
    ap.add_argument("--no-ptrans", action="store_true")
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
    log(f"[bench] n={n} nb={nb} steps={K} warmup={W} free={free / 2**30:.1f} GiB")

    A0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    inputs.fill_matrix_(A0, args.seed)
    B0 = torch.empty((n, args.nrhs), dtype=torch.float64, device=dev)
    inputs.fill_rhs_(B0, args.seed)
    work = lp.workspace(n, nb, "fp64", dev)
    swork = torch.empty(lp.lib.lu_solve_workspace_bytes(n, lp.FP64, args.nrhs), dtype=torch.uint8,
                        device=dev)
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

    A = torch.empty_like(A0)
    X = torch.empty_like(B0)
    for w in range(W):
        A.copy_(A0)
        X.copy_(B0)
        lp.lu_factor(A, nb, "fp64", work=work, ipiv=ipiv, info=info, lookahead=look,
                     panel_cus=args.panel_cus, panel_rows=args.panel_rows)
        lp.lu_solve(A, ipiv, info, X, work=swork)
        lp.residual_check(A0, X, B0)
        torch.cuda.synchronize()
        log(f"[bench] warm-up {w + 1}/{W} done")

    outs = [torch.empty((args.nrhs, 5), dtype=torch.float64, device=dev) for _ in range(K)]
    infos = [torch.empty(1, dtype=torch.int32, device=dev) for _ in range(K)]
    profs = []
    step_s = []
    for i in range(K):
        A.copy_(A0)  # restore the input: outside the timed interval
        X.copy_(B0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, prof = lp.lu_factor(A, nb, "fp64", work=work, ipiv=ipiv, info=infos[i],
                                  lookahead=look, profile=True, panel_cus=args.panel_cus,
                                  panel_rows=args.panel_rows)
        lp.lu_solve(A, ipiv, infos[i], X, work=swork)
        lp.residual_check(A0, X, B0, out=outs[i])
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        profs.append(prof)
        log(f"[bench] step {i + 1}/{K}: {1e3 * step_s[-1]:.1f} ms")
    elapsed = sum(step_s)
    log(f"[bench] timed {K} steps: {elapsed:.3f} s")
    x_head = X.clone()

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
              ("gemm_ms", "panel_ms", "swap_ms", "trsm_ms", "swap_left_ms")}
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
        "step_times": stats_ms(step_s),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 blocked LU with partial pivoting + solve + residual "
                               f"check, n={n}, nb={nb}, nrhs={args.nrhs}, A and b "
                               f"uniform[-0.5,0.5) seed {args.seed}, unshifted",
                   "n": n, "nb": nb, "nrhs": args.nrhs, "lookahead": look,
                   "panel_cus": args.panel_cus, "panel_rows": args.panel_rows},
        "frac_fp64_peak": value / PEAK_FP64_TFLOPS,
        "scaled_residual_max": s_max,
        "backward_error_scaled_residual": s_max,
        "residual_pass": bool(info_ok and s_max < 16.0),
        "roofline": {"kernel": "dgemm_trailing_update", "bound": "mfma",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic_from_profile("gemm.hip", n, nb),
                     "algorithmic_bytes_per_launch": sum(p["gemm_bytes"] for p in profs) /
                     max(gemm_launches, 1)},
        "phases_ms_per_step": phases,
    }
    del A, A0, X
    torch.cuda.empty_cache()
    g_head = load_golden(n, args.seed)
    if g_head is not None:
        line["forward_error_vs_oracle"] = forward_error(x_head, g_head["x"])
    if not args.no_parity and args.parity_n != n:
        log(f"[bench] x-parity n={args.parity_n} against the stored oracle solution ...")
        line["x_parity"] = bench_x_parity(lp, inputs, torch, dev, args.parity_n,
                                          args.parity_nb, args.seed)
    R = max(1, args.mixed_reps)
    if not args.no_mixed:
        mn = args.mixed_n or n
        mnb = args.mixed_nb or nb
        log(f"[bench] mixed {args.mixed_prec} n={mn} nb={mnb} shift={mn} ...")
        line["mixed_ir"] = bench_mixed(lp, inputs, torch, dev, mn, mnb, args.mixed_prec,
                                       float(mn), args.seed, R, args.nrhs, nopiv_leg=True,
                                       fp64_nb=nb)
        log(f"[bench] mixed done: {line['mixed_ir']['ms_per_solve']:.1f} ms/solve, "
            f"speedup {line['mixed_ir']['speedup_vs_fp64']:.2f}x")
        if not args.no_mixed_unshifted:
            # the unshifted variants at the headline's block size: their
            # binary64 fallback is then the headline's solve
            mnb = args.mixed_unshifted_nb or nb
            same = mn == n and mnb == nb
            log(f"[bench] mixed {args.mixed_prec} n={mn} unshifted ...")
            line["mixed_ir_unshifted"] = bench_mixed(
                lp, inputs, torch, dev, mn, mnb, args.mixed_prec, 0.0, args.seed,
                max(1, R - 1), args.nrhs, fp64_leg=False,
                x_ref=(g_head["x"] if g_head is not None else x_head) if same else None,
                x_ref_label="oracle" if g_head is not None else "fp64_path")
            if same:
                mu = line["mixed_ir_unshifted"]
                mu["fp64_ms_same_system"] = line["step_times"]["median_ms"]
                mu["speedup_vs_fp64"] = mu["fp64_ms_same_system"] / mu["ms_per_solve"]
            log(f"[bench] mixed unshifted done: "
                f"{line['mixed_ir_unshifted']['ms_per_solve']:.1f} ms/solve, fell back "
                f"{line['mixed_ir_unshifted']['fell_back']}")
            # the same unshifted system with binary32 update operands: classical
            # refinement converges there (kappa u_32 < 1) without the fallback
            log(f"[bench] mixed fp32 n={mn} unshifted ...")
            mf = bench_mixed(lp, inputs, torch, dev, mn, mnb, "fp32", 0.0, args.seed,
                             max(1, R - 1), args.nrhs, fp64_leg=False,
                             x_ref=(g_head["x"] if g_head is not None else x_head) if same else None,
                             x_ref_label="oracle" if g_head is not None else "fp64_path")
            if same:
                mf["fp64_ms_same_system"] = line["step_times"]["median_ms"]
                mf["speedup_vs_fp64"] = mf["fp64_ms_same_system"] / mf["ms_per_solve"]
            line["mixed_ir_unshifted_fp32"] = mf
            log(f"[bench] mixed fp32 unshifted done: {mf['ms_per_solve']:.1f} ms/solve, fell back "
                f"{mf['fell_back']}")
        torch.cuda.empty_cache()
    if not args.no_ptrans:
        log(f"[bench] PTRANS n={args.ptrans_n} ...")
        line["ptrans"] = bench_ptrans(lp, inputs, torch, dev, args.ptrans_n, args.seed, 20)
        log(f"[bench] PTRANS done: {line['ptrans']['fp64']['GBps']:.0f} GB/s (binary64)")
    if not args.no_serve:
        fr = [float(v) for v in args.serve_fractions.split(",") if v]
        log(f"[bench] serving: {args.serve_requests} requests per rate ...")
        line["serving"] = bench_serving(lp, inputs, torch, dev, args.serve_requests, args.seed,
                                        args.serve_gib, args.serve_lowp, args.serve_small_n,
                                        args.serve_large_slots, fr, args.serve_burst)
        log(f"[bench] serving done: p50 {line['serving']['p50_ms']:.2f} ms, "
            f"p99 {line['serving']['p99_ms']:.2f} ms at the highest rate")
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
