"""Builds the sanitised test drivers into tests/sanitize/_build/.

oracle_driver_asan: the CPU oracle and a driver calling every entry point,
  compiled by gcc with the address and undefined-behaviour sanitizers.
api_driver_asan: the library's host API (pic_api.cpp) compiled with host-only
  sanitizer instrumentation (its device code as usual), linked with the
  package's other objects from its own build and the C ABI driver.

Run directly (python tests/sanitize/build.py) or through the package build
entry point; the package must have been built first (its objects are reused).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
ORACLE_DRIVER = os.path.join(OUT, "oracle_driver_asan")
API_DRIVER = os.path.join(OUT, "api_driver_asan")

SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)


def build_oracle_driver(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-fopenmp", "-std=c11",
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-o", ORACLE_DRIVER, "-lm"], verbose)
    return ORACLE_DRIVER


def build_api_driver(verbose: bool = False) -> str:
    sys.path.insert(0, ROOT)
    from paper_2508_06771_amd import build as pkg
    os.makedirs(OUT, exist_ok=True)
    api_src = [s for s in pkg.sources() if os.path.basename(s) == "pic_api.cpp"][0]
    others = [pkg.object_of(s) for s in pkg.sources() if s != api_src]
    missing = [o for o in others if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"package objects missing (build the package first): {missing}")
    api_obj = os.path.join(OUT, "pic_api.asan.o")
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    _run(["hipcc", *pkg.HIPCC_FLAGS, *host_san, "-g", "-I", pkg.INCLUDE, "-x", "hip", "-c",
          api_src, "-o", api_obj], verbose)
    drv_obj = os.path.join(OUT, "api_driver.o")
    _run(["/opt/rocm/lib/llvm/bin/clang++", "-O1", "-g", "-std=c++17", *SAN,
          "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", pkg.INCLUDE, "-c",
          os.path.join(HERE, "api_driver.cpp"), "-o", drv_obj], verbose)
    # host link: the objects already carry their gfx950 code objects
    _run(["/opt/rocm/lib/llvm/bin/clang++", *SAN, drv_obj, api_obj, *others,
          "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", API_DRIVER], verbose)
    return API_DRIVER


def build(verbose: bool = False) -> None:
    build_oracle_driver(verbose)
    build_api_driver(verbose)


if __name__ == "__main__":
    build(verbose=True)
