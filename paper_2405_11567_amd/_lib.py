"""ctypes loader for libfsv.so.  There is no fallback: if the library is not
built, every call raises."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsv.so")

FSV_OK = 0
FSV_EINVAL = -1
FSV_ENOMEM = -2
FSV_EDEVICE = -3
FSV_ESTATE = -4
FSV_ENONFINITE = -5
_NAMES = {FSV_EINVAL: "EINVAL", FSV_ENOMEM: "ENOMEM", FSV_EDEVICE: "EDEVICE",
          FSV_ESTATE: "ESTATE", FSV_ENONFINITE: "ENONFINITE"}


class FsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int32),
        ("n_alpha", ctypes.c_int32),
        ("n_beta", ctypes.c_int32),
        ("ordering", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("h", ctypes.POINTER(ctypes.c_double)),
        ("g", ctypes.POINTER(ctypes.c_double)),
        ("e_core", ctypes.c_double),
        ("n_ops", ctypes.c_int32),
        ("ops", ctypes.POINTER(ctypes.c_int32)),
        ("excitation", ctypes.c_int32),
    ]


EXPORTS = [
    "fsv_last_error", "fsv_plan_create", "fsv_plan_destroy", "fsv_state_bytes", "fsv_plan_info",
    "fsv_plan_workspace_bytes", "fsv_plan_device_bytes", "fsv_plan_set_workspace", "fsv_batch_arena_bytes",
    "fsv_plan_set_engine", "fsv_plan_runs", "fsv_time_runs",
    "ansatz_apply", "energy", "energy_grad", "energy_grad_noalloc", "energy_grad_fd", "rdm1",
    "set_onebody_potential",
    "fsv_set_theta", "fsv_forward_async", "fsv_sigma_async", "fsv_reverse_async", "fsv_finish",
    "fsv_autotune", "fsv_batch_create", "fsv_batch_destroy", "fsv_batch_energy_grad",
    "fsv_batch_bytes", "fsv_batch_autotune", "fsv_batch_set_initial_state", "fsv_pool_create", "fsv_pool_destroy", "fsv_pool_gradients",
    "fsv_set_initial_state", "onebody_expectation",
]

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2405_11567_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    c_int = ctypes.c_int
    lib.fsv_last_error.restype = ctypes.c_char_p
    lib.fsv_last_error.argtypes = []
    lib.fsv_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Problem), vp]
    lib.fsv_plan_destroy.argtypes = [vp]
    lib.fsv_state_bytes.restype = ctypes.c_size_t
    lib.fsv_state_bytes.argtypes = [vp]
    lib.fsv_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_uint64)]
    for name in ("fsv_plan_workspace_bytes", "fsv_plan_device_bytes", "fsv_batch_arena_bytes"):
        getattr(lib, name).restype = ctypes.c_size_t
        getattr(lib, name).argtypes = [vp]
    lib.fsv_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    lib.fsv_plan_set_engine.argtypes = [vp, c_int]
    lib.fsv_plan_runs.argtypes = [vp, c_int, i32, i32]
    lib.fsv_time_runs.argtypes = [vp, c_int, vp, vp, ctypes.POINTER(ctypes.c_float)]
    lib.ansatz_apply.argtypes = [vp, d, vp]
    lib.energy.argtypes = [vp, vp, d]
    lib.energy_grad.argtypes = [vp, vp, vp, vp, d, vp]  # theta and grad as addresses (the hot call)
    lib.energy_grad_noalloc.argtypes = [vp, d, vp, vp, d, d]
    lib.energy_grad_fd.argtypes = [vp, d, ctypes.c_double, vp, d, d]
    lib.rdm1.argtypes = [vp, vp, d]
    lib.set_onebody_potential.argtypes = [vp, d]
    lib.fsv_set_theta.argtypes = [vp, d]
    lib.fsv_forward_async.argtypes = [vp, vp]
    lib.fsv_sigma_async.argtypes = [vp, vp, vp]
    lib.fsv_reverse_async.argtypes = [vp, vp, vp]
    lib.fsv_finish.argtypes = [vp, d, d]
    lib.fsv_autotune.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_char_p)]
    lib.fsv_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Problem), ctypes.c_int32, vp]
    lib.fsv_batch_destroy.argtypes = [vp]
    lib.fsv_batch_energy_grad.argtypes = [vp, d, vp, d, d]
    lib.fsv_batch_bytes.restype = ctypes.c_size_t
    lib.fsv_batch_bytes.argtypes = [vp]
    lib.fsv_batch_autotune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_char_p)]
    lib.fsv_batch_set_initial_state.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), d]
    lib.fsv_pool_create.argtypes = [ctypes.POINTER(vp), vp, i32, ctypes.c_int32, ctypes.c_int32]
    lib.fsv_pool_destroy.argtypes = [vp]
    lib.fsv_pool_gradients.argtypes = [vp, d, vp, vp, d, d]
    lib.fsv_set_initial_state.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), d]
    lib.onebody_expectation.argtypes = [vp, vp, d, d]
    for name in EXPORTS:
        if name not in ("fsv_last_error", "fsv_state_bytes", "fsv_batch_bytes", "fsv_plan_workspace_bytes",
                        "fsv_plan_device_bytes", "fsv_batch_arena_bytes"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def check(rc: int):
    if rc != FSV_OK:
        msg = load().fsv_last_error()
        raise FsvError(rc, msg.decode() if msg else "")
