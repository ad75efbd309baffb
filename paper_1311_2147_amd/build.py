"""Builds libbcinc.so (HIP for gfx950) in-tree with hipcc, and the CPU
comparator's libcpu_incremental.so with gcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libbcinc.so")
SOURCES = [os.path.join(CSRC, "bcinc.hip")]
DEPENDS = [os.path.join(CSRC, f) for f in ("bc_device.h", "bc_kernels.hip", "bc_check.hip", "bc_host.hip", "bcinc.hip")] + [
    os.path.join(os.path.dirname(HERE), "include", "bcinc.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed fp32 instructions stay off (the compiler is told the target lacks them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the process shares PyTorch's HIP runtime (see bcinc.py); v5 code objects load on every ROCm 6/7 runtime
    "-mcode-object-version=5",
    "-Wall", "-Wno-unused-function",
]


CPU_SRC = os.path.join(HERE, "cpu", "cpu_incremental.c")
CPU_LIB = os.path.join(HERE, "cpu", "libcpu_incremental.so")


def build_cpu(verbose: bool = False) -> str:
    cmd = [os.environ.get("CC", "gcc"), "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", CPU_SRC, "-o",
           CPU_LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed:\n" + res.stdout + res.stderr)
    if verbose and (res.stdout or res.stderr):
        print(res.stdout + res.stderr)
    os.replace(CPU_LIB + ".tmp", CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False) -> str:
    build_cpu(verbose)
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", LIB_PATH + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and (res.stdout or res.stderr):
        print(res.stdout + res.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
