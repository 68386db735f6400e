"""Build libvp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2605_21794_amd.build

Flags: -O3, gfx950 only, no floating-point contraction (the float64 push then follows the
plain definition's rounding step by step), packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libvp.so")
SOURCES = ["vp_kernels.hip", "vp_cluster.hip", "vp_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source into libvp.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra or []) + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


def emit_asm(out_dir: str) -> list:
    """Write the gfx950 assembly of the kernels (for inspection of our own code)."""
    os.makedirs(out_dir, exist_ok=True)
    src = os.path.join(CSRC, "vp_kernels.hip")
    cmd = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
        "--cuda-device-only", "-S", src, "-o", os.path.join(out_dir, "vp_kernels.s")]
    subprocess.run(cmd, check=True)
    return [os.path.join(out_dir, "vp_kernels.s")]


if __name__ == "__main__":
    print(build(verbose=True))
