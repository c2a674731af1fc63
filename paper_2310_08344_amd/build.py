"""Builds the HIP library ``_lx.so`` in-tree for gfx950.

    python -m paper_2310_08344_amd.build [--jobs N]

Host sources are compiled as plain C++ by the ROCm clang, the kernels as HIP
for gfx950; packed-FP32 instruction selection is switched off for the device
code.  Objects go to ``_build/`` next to the package; the shared object is
written next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "_lx.so")
ARCH = "gfx950"

HIP_SOURCES = ["kernels.hip", "pair.hip", "block.hip", "stream.hip", "batch.hip", "mlp.hip", "static_ws.hip"]
CXX_SOURCES = ["lx_api.cpp", "lx_batch.cpp", "lx_predictor.cpp", "planner.cpp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _common() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _compile(cmd: list[str]) -> None:
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + res.stdout)
    if res.stdout.strip():
        # keep compiler warnings visible, without the host pass's note about
        # the device-only target feature
        lines = [ln for ln in res.stdout.splitlines() if "packed-fp32-ops" not in ln]
        if any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")


def build(jobs: int = 4, verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *_common(),
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append([hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *_common(),
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(_compile, cmds))
    tmp = LIB + ".tmp"
    _compile([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    build(args.jobs, verbose=True)


if __name__ == "__main__":
    main()
