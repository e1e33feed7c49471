"""Builds tests/host_sanitize/_build/host_abi_check: the library's host layer
(csrc/tlda_api.hip) compiled with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code only (device code is built as
usual), linked with the library's other objects and the check driver
host_abi_check.cpp.  Needs the objects of the library build
(paper_2511_07809_amd/build.py), which __graft_entry__.build() runs first.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "host_abi_check")

sys.path.insert(0, ROOT)
from paper_2511_07809_amd import build as lib_build  # noqa: E402

# host-side instrumentation only: every sanitizer flag applies to the host
# compilation of the HIP source
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = "-fsanitize=address,undefined"
DRIVER_FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", SAN,
                "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
                "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = sorted(os.path.join(lib_build.BUILD, f) for f in os.listdir(lib_build.BUILD)
                  if f.endswith(".o") and f != "tlda_api.o")
    if not objs:
        raise RuntimeError("library objects missing: run paper_2511_07809_amd/build.py first")
    api = os.path.join(OUT, "tlda_api_san.o")
    _run([lib_build._hipcc(), *lib_build.HIPCC_FLAGS, *HOST_SANITIZE, "-c",
          os.path.join(lib_build.CSRC, "tlda_api.hip"), "-o", api])
    drv = os.path.join(OUT, "host_abi_check.o")
    _run([CLANG, *DRIVER_FLAGS, "-c", os.path.join(HERE, "host_abi_check.cpp"), "-o", drv])
    _run([CLANG, SAN, "-o", EXE, drv, api, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib"])
    if verbose:
        print(f"built {EXE}")
    return EXE


if __name__ == "__main__":
    build(verbose=True)
