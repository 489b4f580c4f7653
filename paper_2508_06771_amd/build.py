"""Builds libpiccoll.so (HIP for gfx950) in the package directory.

Each source compiles to its own object in parallel (kernels and their launch
code live in the same translation unit, so no relocatable device code is
needed), then one link step makes the shared library.  The objects stay in
`_build/` beside the sources, so other links (the host-sanitised test
driver) can reuse them.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpiccoll.so")
OBJ_DIR = os.path.join(PKG, "_build")
INCLUDE = os.path.join(ROOT, "include")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed-FP32 instructions are emitted (only scalar / float2 code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip"))) + \
        sorted(glob.glob(os.path.join(PKG, "csrc", "*.cpp")))


def object_of(src: str) -> str:
    return os.path.join(OBJ_DIR, os.path.basename(src) + ".o")


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", INCLUDE, "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libpiccoll.so (always recompiles)."""
    srcs = sources()
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [object_of(s) for s in srcs]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_compile, s, o, verbose) for s, o in zip(srcs, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
