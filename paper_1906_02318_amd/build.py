"""Builds libmpmi.so (the C-ABI library) in-tree with hipcc for gfx950.

Usage: python -m paper_1906_02318_amd.build   (or call build()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpmi.so")
SOURCES = ["mpmi_abi.cpp", "mpmi_tick.hip", "mpmi_fit.hip", "mpmi_multi.hip", "mpmi_mlp.hip", "mpmi_bf16.hip", "mpmi_split.hip", "mpmi_diag.hip", "mpmi_lifted.hip", "mpmi_recheck64.hip", "mpmi_select.hip"]
HEADERS = ["mpmi_device.hpp", "mpmi_launch.hpp", "mpmi_tick_common.hpp"]

ARCH = os.environ.get("MPMI_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Packed FP32 instructions are kept out of every kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _dynamic_stack_kernels(remarks: str) -> list:
    """Kernels the compiler reports with a dynamic stack (a device call whose
    depth it cannot bound, e.g. recursion): their private segment can overflow."""
    bad, name = [], None
    for line in remarks.splitlines():
        if "remark: Function Name:" in line:
            name = line.split("Function Name:", 1)[1].split("[-Rpass")[0].strip()
        elif "remark:     Dynamic Stack: True" in line and name:
            bad.append(name)
    return bad


def _compile(src: str) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    if src.endswith(".hip"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    bad = _dynamic_stack_kernels(r.stderr)
    if bad:
        raise RuntimeError(f"{src}: device code with a dynamic stack (unbounded device calls): {bad}")
    return out


def build(verbose: bool = False) -> str:
    """Compiles every source (always) and links libmpmi.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
