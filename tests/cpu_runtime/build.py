"""Build the host-check variant of libfsv: the library's own sources, host code
instrumented with AddressSanitizer and UndefinedBehaviorSanitizer, linked
against the host-only HIP stand-in (hip_stub.cpp) instead of the HIP runtime.
Test infrastructure only: kernels never run in this build.

Outputs (under tests/cpu_runtime/_build): libhipstub.so, libfsv_hostcheck.so.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2405_11567_amd import build as pkg_build  # noqa: E402

OUT = os.path.join(HERE, "_build")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = pkg_build.HIPCC
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime (to preload into Python)."""
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        raise RuntimeError("clang's AddressSanitizer runtime is not installed")
    return cands[-1]


def paths():
    return os.path.join(OUT, "libhipstub.so"), os.path.join(OUT, "libfsv_hostcheck.so")


def build(verbose: bool = False) -> tuple:
    os.makedirs(OUT, exist_ok=True)
    stub, lib = paths()

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    run([CLANG, "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address", "-shared-libasan",
         "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         os.path.join(HERE, "hip_stub.cpp"), "-o", stub])
    objs = []
    for src in pkg_build.SOURCES:
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        flags = [f for f in pkg_build.FLAGS if f != "-O3"]
        run([HIPCC, *flags, "-O1", "-g", *SAN, "-c", os.path.join(pkg_build.CSRC, src), "-o", obj])
        objs.append(obj)
    run([CLANG, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libasan", "-o", lib, *objs,
         "-L" + OUT, "-lhipstub", "-Wl,-rpath," + OUT])
    return stub, lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
