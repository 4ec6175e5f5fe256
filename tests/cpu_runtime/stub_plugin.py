"""pytest plugin: run the GPU test files on the CPU against a checking build
of the library (tests/cpu_runtime/build.py), so that their exact sequence of
plan / pool / batch lifetimes, calls, oracle calls and garbage collections
runs under AddressSanitizer.

* Default: the host-check build.  Kernels do not run, so results are
  meaningless: use it with
  `python -O -m pytest --assert=plain -p tests.cpu_runtime.stub_plugin ...`,
  which strips the tests' assertions.
* FSV_STUB_LIB=kexec: the kernel-executing build.  Kernels run on the host,
  so results are real and the tests' assertions stay on.

States are CPU tensors over buffers of the stand-in's device allocator.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import types

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")


def pytest_configure(config):
    import torch

    import paper_2405_11567_amd as fsv
    from paper_2405_11567_amd import _lib

    ctypes.CDLL(os.path.join(BUILD, "libhipstub.so"), mode=ctypes.RTLD_GLOBAL)
    kexec = os.environ.get("FSV_STUB_LIB") == "kexec"
    _lib.LIB_PATH = os.path.join(BUILD, "libfsv_kexec.so" if kexec else "libfsv_hostcheck.so")
    _lib._lib = None

    cuda = types.SimpleNamespace(
        is_available=lambda: True,
        device=lambda *_: contextlib.nullcontext(),
        current_stream=lambda *_: types.SimpleNamespace(cuda_stream=0),
        synchronize=lambda *_: None,
    )

    class TorchShim:
        def __getattr__(self, name):
            if name == "cuda":
                return cuda
            if name == "device":
                return lambda *a, **k: torch.device("cpu")
            return getattr(torch, name)

    shim = TorchShim()
    fsv._torch = lambda: shim

    # states come from the stand-in's device allocator, so that its copy and
    # GEMM checks cover them; the tensor frees its buffer when it dies
    import weakref
    stub = ctypes.CDLL(os.path.join(BUILD, "libhipstub.so"))
    stub.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    stub.hipFree.argtypes = [ctypes.c_void_p]

    import numpy as np

    def stub_tensor(nbytes, dtype):
        p = ctypes.c_void_p()
        if stub.hipMalloc(ctypes.byref(p), max(nbytes, 1)) != 0:
            raise MemoryError("stand-in hipMalloc failed")
        buf = (ctypes.c_char * max(nbytes, 1)).from_address(p.value)
        # the buffer is freed when the last tensor or array over it is gone
        # (every view keeps this array alive through its storage)
        arr = np.frombuffer(buf, dtype=np.uint8)
        weakref.finalize(arr, stub.hipFree, p.value)
        return torch.from_numpy(arr).view(dtype)

    def new_state(self):
        return stub_tensor((1 << self.n_qubits) * (16 if self.precision == 0 else 8), self.dtype)

    fsv.Plan.new_state = new_state
    fsv._device_buffer = lambda device, nbytes: stub_tensor(int(nbytes), torch.uint8)

    # the oracle: its AddressSanitizer build when one is present
    asan_oracle = os.environ.get("FSV_ORACLE_LIB")
    if asan_oracle:
        from oracle import sector
        sector._LIB = asan_oracle
        sector.build = lambda force=False: asan_oracle



def pytest_sessionstart(session):
    import sys
    for mod in list(sys.modules.values()):
        if getattr(mod, "gpu_available", None) is not None and mod.__name__.endswith("conftest"):
            mod.gpu_available = lambda: True


def pytest_collection_modifyitems(config, items):
    # FSV_STUB_RUN_SKIPPED=1: also replay tests that are skipped on the GPU
    if os.environ.get("FSV_STUB_RUN_SKIPPED"):
        for it in items:
            it.own_markers = [m for m in it.own_markers if m.name != "skip"]
