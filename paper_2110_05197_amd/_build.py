"""Build libmclbm.so (HIP for gfx950) in-tree with hipcc.

Each translation unit compiles in its own hipcc process (in parallel), then
they are linked into ``paper_2110_05197_amd/libmclbm.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmclbm.so")
PROBE = os.path.join(PKG, "stream_probe")
SOURCES = ["mclbm.hip", "inst_p0.hip", "inst_p1.hip", "inst_p2.hip", "inst_p3.hip"]
ARCH = os.environ.get("MCLBM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # contraction decided per source expression: identical arithmetic in every
    # kernel that inlines the same node function (fused, two-pass, batched)
    "-ffp-contract=on",
    # no packed FP32 instructions (v_pk_*_f32) in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no mixed-precision FMA (v_fma_mix*): folding "fma in FP32, then round
    # to FP16" into one instruction rounds once instead of twice, so the
    # kernels that happened to get the fold would differ from the others by
    # an FP16 ulp at ties
    "-Xclang", "-target-feature", "-Xclang", "-fma-mix-insts",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc", "-c", *FLAGS, "-o", obj, os.path.join(CSRC, src)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "unknown target feature" not in l
                    and "packed-fp32-ops" not in l and "fma-mix-insts" not in l
                    and l.strip() not in ("1 warning generated.", "2 warnings generated."))
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj


def _build_probe() -> str:
    """The stream-pattern bandwidth probe (measurement only, not the library)."""
    cmd = ["hipcc", *[f for f in FLAGS if f != "-fPIC"], "-o", PROBE + ".tmp",
           os.path.join(CSRC, "stream_probe.hip")]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for stream_probe.hip:\n{r.stdout}")
    os.replace(PROBE + ".tmp", PROBE)
    return PROBE


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES) + 1, max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(jobs) as ex:
        probe = ex.submit(_build_probe)
        objs = list(ex.map(_compile, SOURCES))
        probe.result()
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, "and", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
