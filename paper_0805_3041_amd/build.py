"""Builds libmg.so (the HIP library behind include/mg.h) in-tree for gfx950.

    python -m paper_0805_3041_amd.build

Every call compiles from source.  The library is written for gfx950 only.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmg.so")
SOURCES = ["mg_kernels.hip", "mg_fused.hip", "mg_api.hip", "mg_tune.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no FMA contraction: a node gets bit-identical values from every kernel
    # that can update it (tile passes, per-op kernels, coarse interpreter)
    "-ffp-contract=off",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    # packed FP32 ops are kept off the device code path
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the first kernel arguments (level-descriptor pointers, tile shape)
    # arrive preloaded in SGPRs: a launch's first descriptor load need not
    # wait for a kernarg load (about 1 % per cycle with ~50 launches)
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def flags_key() -> str:
    """The compile flags that shape the device code (include paths left out)."""
    out, skip = [], False
    for f in FLAGS:
        if skip:
            skip = False
            continue
        if f == "-I":
            skip = True
            continue
        out.append(f)
    return " ".join(out)


def source_digest() -> str:
    """sha256 (first 16 hex digits) over the compile flags and the kernel
    sources and headers: the autotuner's cached choices are keyed by it."""
    import hashlib

    d = hashlib.sha256(flags_key().encode() + b"\0")
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                d.update(name.encode() + b"\0" + f.read())
    return d.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, f'-DMG_SOURCE_DIGEST="{source_digest()}"', "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    print("built", LIB)
