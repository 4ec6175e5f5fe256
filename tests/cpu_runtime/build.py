"""Build the checking variants of libfsv against the host-only HIP stand-in
(hip_stub.cpp) instead of the HIP runtime, instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer.  Test infrastructure only.

* libfsv_hostcheck.so: the library's sources compiled by hipcc; host code
  runs, kernels do not.
* libfsv_kexec.so: the same sources compiled as plain C++ against
  kexec/hip/hip_runtime.h, so that kernels run on the host too (one thread
  per work-item) and every memory access they make is checked.  The only
  change to the sources is mechanical: a dynamic LDS declaration
  (`extern __shared__ T name[];`) becomes a pointer to the launch's LDS block.

Outputs (under tests/cpu_runtime/_build): libhipstub.so, libfsv_hostcheck.so,
libfsv_kexec.so.
"""

from __future__ import annotations

import glob
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

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


def kexec_path():
    return os.path.join(OUT, "libfsv_kexec.so")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_stub(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    stub = paths()[0]
    _run([CLANG, "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address", "-shared-libasan",
          "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          os.path.join(HERE, "hip_stub.cpp"), "-o", stub, "-lpthread"], verbose)
    return stub


_DYN_LDS = re.compile(r"extern __shared__ (\w+) (\w+)\[\];")


def build_kexec(verbose: bool = False, csrc_dir: str | None = None) -> str:
    """The kernel-executing build (see the module docstring); csrc_dir: another
    copy of the kernel sources to build instead of the package's."""
    build_stub(verbose)
    src_root = os.path.join(OUT, "kexec_src")
    csrc = os.path.join(src_root, "paper_2405_11567_amd", "csrc")
    os.makedirs(csrc, exist_ok=True)
    os.makedirs(os.path.join(src_root, "include"), exist_ok=True)
    shutil.copy(os.path.join(ROOT, "include", "fsv.h"), os.path.join(src_root, "include", "fsv.h"))
    src = csrc_dir or pkg_build.CSRC
    for name in os.listdir(src):
        if name.endswith((".hip", ".h")):
            text = open(os.path.join(src, name)).read()
            text = _DYN_LDS.sub(lambda m: f"{m.group(1)} *{m.group(2)} = ({m.group(1)} *)fsv_cpu_dyn_lds();", text)
            open(os.path.join(csrc, name), "w").write(text)
    flags = ["-x", "c++", "-std=c++17", "-O1", "-g", "-fPIC", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(HERE, "kexec"), "-I/opt/rocm/include", "-Wno-unused-command-line-argument"]

    def one(src):
        obj = os.path.join(OUT, "kexec_" + src.replace(".hip", ".o"))
        _run([CLANG, *flags, "-c", os.path.join(csrc, src), "-o", obj], verbose)
        return obj

    with ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(one, pkg_build.SOURCES))
    lib = kexec_path()
    _run([CLANG, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libasan", "-o", lib, *objs,
          "-L" + OUT, "-lhipstub", "-Wl,-rpath," + OUT, "-lpthread"], verbose)
    return lib


def build(verbose: bool = False) -> tuple:
    os.makedirs(OUT, exist_ok=True)
    stub, lib = paths()

    def run(cmd):
        _run(cmd, verbose)

    build_stub(verbose)
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
    if "kexec" in sys.argv:
        other = [a for a in sys.argv[1:] if a not in ("kexec", "-v")]
        print(build_kexec(verbose="-v" in sys.argv, csrc_dir=other[0] if other else None))
    else:
        print(build(verbose="-v" in sys.argv))
