"""Builds libhacc_sr.so (all HIP sources of csrc/) for gfx950 with hipcc.

Flags: -O3, no fast-math and no floating-point contraction (the kernels
write every fused multiply-add explicitly and rely on exact float32
rounding in their compensated sums), packed-FP32 instructions disabled.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhacc_sr.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else (shutil.which("hipcc") or "hipcc")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def hashed_files():
    """Every file the library is compiled from: the HIP sources, the internal
    header and the public header."""
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) +
                  glob.glob(os.path.join(CSRC, "*.h"))) + [
        os.path.join(INCLUDE, "hacc_sr.h")]


def source_hash() -> str:
    """sha256 over the names and exact bytes of the files in hashed_files().
    The build embeds it in the library (hacc_sr_source_hash), and the binding
    refuses a library whose embedded hash differs from the sources in the
    tree, so a stale build never runs."""
    import hashlib
    h = hashlib.sha256()
    for path in hashed_files():
        h.update(os.path.relpath(path, ROOT).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    """Compile every csrc/*.hip into one shared library and return its path."""
    tag = os.path.splitext(os.path.basename(out))[0]
    build_dir = os.path.join(os.path.dirname(out), "_build", tag)
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    tag_flag = f'-DHSR_SOURCE_SHA256="{source_hash()}"'
    for src in sources():
        obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
        cmd = [hipcc(), *HIP_FLAGS, *extra_flags, tag_flag, "-I", INCLUDE,
               "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
