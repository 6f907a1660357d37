"""Builds liblp.so (the gfx950 kernels + C ABI) and the input generator library.

    python -m paper_2202_13995_amd.build        # compile everything

Each .hip file is compiled with hipcc for gfx950 only; packed FP32 instructions
are disabled for the device code.  Objects go to paper_2202_13995_amd/_build/,
the shared libraries next to the sources that load them.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblp.so")
GEN_SRC = os.path.join(ROOT, "inputs", "gen.hip")
GEN_LIB = os.path.join(ROOT, "inputs", "libinputs_gen.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]
SOURCES = ["gemm.hip", "gemm_lp.hip", "panel.hip", "panel_fused.hip", "nopiv.hip", "ptrans.hip", "solve.hip",
           "driver.hip", "ir.hip", "serve.hip"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the device-only feature flag: not an error
    err = "\n".join(ln for ln in r.stderr.splitlines()
                    if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{err}")
    return err


def _compile(src: str, obj: str):
    return _run([HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])


def _stale(src: str, obj: str) -> bool:
    """True when obj is missing or older than src or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "lp.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source (always, so the build check is real), or with
    incremental=True only those whose object is older than the sources."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(BUILD, s.replace(".hip", ".o")) for s in srcs]
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    gen_obj = os.path.join(BUILD, "inputs_gen.o")
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, 16))) as ex:
        futs = [ex.submit(_compile, os.path.join(CSRC, s), o) for s, o in zip(srcs, objs)
                if not incremental or _stale(os.path.join(CSRC, s), o)]
        if not incremental or _stale(GEN_SRC, gen_obj):
            futs.append(ex.submit(_compile, GEN_SRC, gen_obj))
        for f in futs:
            msg = f.result()
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    tmp = GEN_LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, gen_obj])
    os.replace(tmp, GEN_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
