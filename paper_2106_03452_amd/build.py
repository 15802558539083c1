"""Build ``libpsr.so`` (the C-ABI solver library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpsr.so")
SOURCES = ["psr_kernels.hip", "psr_mc.hip", "psr_opt.hip", "psr_slab.hip", "psr_api.cpp"]
ARCH = os.environ.get("PSR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libpsr.so)")


def compile_command(out: str, defines: tuple[str, ...] = ()) -> list[str]:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed-FP32 instructions stay off in every HIP object of this library
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", INCLUDE, "-I", CSRC, "-o", out,
    ] + [f"-D{d}" for d in defines] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, out: str = LIB, defines: tuple[str, ...] = ()) -> str:
    """Compile the library (always recompiles) and return its path."""
    tmp = out + ".tmp"
    cmd = compile_command(tmp, defines)
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError(f"hipcc failed with exit code {proc.returncode}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
