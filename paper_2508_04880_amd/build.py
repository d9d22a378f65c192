"""Build ``libtusq.so`` in-tree: HIP sources with hipcc for gfx950, host
sources with g++, linked by hipcc.  Usage: ``python -m paper_2508_04880_amd.build``.
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
LIB = os.path.join(PKG, "libtusq.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_SOURCES = ["kernels.hip", "exec.hip", "batch.hip"]
CXX_SOURCES = ["host_ecm.cpp", "host_plan.cpp", "capi.cpp", "serve.cpp"]

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # keep hipcc from forming packed FP32 instructions
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # keep the register-blocked sweep's amplitude array in registers:
             # merging near-identical switch cases would address it through
             # pointer phis and move it to scratch memory
             "-mllvm", "-simplifycfg-sink-common=false",
             "-Wall", "-Wno-unused-result"]
# per-source additions: the sweep kernels' and the batched walk's program
# dispatch branches on wave-uniform instruction words only, so its control
# flow needs no structurizing; structurized, every lane exchange (an
# in-place permlane / DPP swap) first copied the whole register tile, and
# the batched register programs held 220 VGPRs instead of 140
HIP_SOURCE_FLAGS = {"kernels.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions"],
                    "batch.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions"]}
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
             # complex products by the plain formula: the same values for
             # finite operands, without a library call per product
             "-fcx-limited-range",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-pthread"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    jobs = []
    for s in HIP_SOURCES:
        if os.path.exists(os.path.join(CSRC, s)):
            jobs.append([hipcc, *HIP_FLAGS, *HIP_SOURCE_FLAGS.get(s, []), f"-I{INCLUDE}", f"-I{CSRC}", "-c",
                         os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o")])
    for s in CXX_SOURCES:
        if os.path.exists(os.path.join(CSRC, s)):
            jobs.append(["g++", *CXX_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c",
                         os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o")])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o, file=sys.stderr)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
