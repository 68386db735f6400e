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
# (source, object name, extra defines): the fused step is compiled once per precision mode
SOURCES = [("vp_kernels.hip", "vp_kernels", []), ("vp_persist.hip", "vp_persist", []),
           ("vp_cluster.hip", "vp_cluster", []), ("vp_api.cpp", "vp_api", [])] + [
    ("vp_fused.hip", f"vp_fused_{m}", [f"-DVP_FUSED_MODE={m}"]) for m in range(4)]
# every file whose text the kernels are built from
KERNEL_SOURCES = ["vp_device.h", "vp_internal.h", "vp_kernels.hip", "vp_fused.hip", "vp_persist.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source into libvp.so (always recompiles): one object per source,
    compiled side by side, then linked."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile
    compile_flags = [f for f in FLAGS if f != "-shared"] + list(extra or [])
    with tempfile.TemporaryDirectory(prefix="vp_build_") as tmpdir:
        objs, cmds = [], []
        for src, name, defs in SOURCES:
            obj = os.path.join(tmpdir, name + ".o")
            objs.append(obj)
            cmds.append([HIPCC] + compile_flags + defs + ["-c", os.path.join(CSRC, src), "-o", obj])
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([HIPCC] + FLAGS + list(extra or []) + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    return LIB


def emit_asm(out_dir: str) -> list:
    """Write the gfx950 assembly of the kernels (for inspection of our own code)."""
    os.makedirs(out_dir, exist_ok=True)
    outs = []
    for src, name, defs in SOURCES:
        if not src.endswith(".hip"):
            continue
        out = os.path.join(out_dir, name + ".s")
        cmd = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + defs + [
            "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
        subprocess.run(cmd, check=True)
        outs.append(out)
    return outs


if __name__ == "__main__":
    print(build(verbose=True))
