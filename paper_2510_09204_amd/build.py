"""Build the SF shared library (libsf.so) for gfx950 with hipcc, in-tree.

Usage:  python -m paper_2510_09204_amd.build [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
INCLUDE = PKG.parent / "include"
LIB = PKG / "libsf.so"
SOURCES = [CSRC / "sf_kernels.hip", CSRC / "sf_kernels3d.hip", CSRC / "sf_select.hip",
           CSRC / "sf_host.cpp"]

# Packed FP32 instructions stay off: the compiler would otherwise form
# v_pk_* FP32 ops from scalar and float2 code.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
             f"-I{INCLUDE}", f"-I{CSRC}"]


def source_digest() -> str:
    """SHA-256 over the library's sources (kernels, internal header, host
    runtime, public header): identifies the kernels a measurement was taken
    on."""
    import hashlib
    h = hashlib.sha256()
    for f in (*SOURCES, CSRC / "sf_internal.h", INCLUDE / "sf.h"):
        h.update(f.name.encode())
        h.update(f.read_bytes())
    return h.hexdigest()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> Path:
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), *HIP_FLAGS, *map(str, SOURCES), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    if verbose and res.stderr.strip():
        # the host pass warns about the device-only target feature
        lines = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
        if any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
