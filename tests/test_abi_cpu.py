"""C-ABI checks that need no GPU: the library loads, exports every function
that include/fsv.h declares, and rejects invalid problems before touching the
device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_11567_amd import _lib
    return _lib.load()


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert "energy_grad" in names and "fsv_plan_create" in names and len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    from paper_2405_11567_amd import _lib
    assert sorted(_lib.EXPORTS) == names


def _problem(n=8, na=2, nb=2, ops=None, h=None, g=None, ordering=0, precision=0):
    from paper_2405_11567_amd import _lib
    from workloads import random_problem
    p = random_problem(n, na + nb, None, seed=3)
    h = p.h if h is None else h
    g = p.g if g is None else g
    ops = p.ops if ops is None else np.asarray(ops, dtype=np.int32).reshape(-1, 4)
    keep = [np.ascontiguousarray(h, dtype=np.float64), np.ascontiguousarray(g, dtype=np.float64),
            np.ascontiguousarray(ops, dtype=np.int32)]
    cp = _lib.Problem(n, na, nb, ordering, precision,
                      keep[0].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      keep[1].ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0,
                      keep[2].shape[0], keep[2].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return cp, keep


@pytest.mark.parametrize("kw,code", [
    (dict(n=7), -1), (dict(n=36), -1), (dict(na=5), -1), (dict(ordering=2), -1),
    (dict(precision=3), -1), (dict(ops=[[0, 2, 1, 3]]), -1), (dict(ops=[[2, 2, 0, 1]]), -1),
    (dict(ops=[[2, -1, -1, 1]]), -1), (dict(ops=[[2, -1, 3, 0]]), -1), (dict(ops=[[16, -1, -1, 0]]), -1),
])
def test_invalid_problem_rejected(lib, kw, code):
    cp, keep = _problem(**kw)
    out = ctypes.c_void_p()
    rc = lib.fsv_plan_create(ctypes.byref(out), ctypes.byref(cp), None)
    assert rc == code
    assert out.value is None
    assert len(lib.fsv_last_error()) > 0


def test_nonfinite_and_asymmetric_integrals(lib):
    from workloads import random_problem
    p = random_problem(8, 4, None, seed=3)
    h = p.h.copy(); h[0, 1] = np.nan
    cp, keep = _problem(h=h)
    out = ctypes.c_void_p()
    assert lib.fsv_plan_create(ctypes.byref(out), ctypes.byref(cp), None) == -5
    g = p.g.copy(); g[0, 1, 2, 3] += 1e-3
    cp, keep = _problem(g=g)
    assert lib.fsv_plan_create(ctypes.byref(out), ctypes.byref(cp), None) == -1
    assert b"symmetry" in lib.fsv_last_error()
    h = p.h.copy(); h[0, 1] += 0.1
    cp, keep = _problem(h=h)
    assert lib.fsv_plan_create(ctypes.byref(out), ctypes.byref(cp), None) == -1


def test_null_arguments(lib):
    assert lib.fsv_plan_create(None, None, None) == -1
    assert lib.fsv_plan_destroy(None) == 0
    assert lib.fsv_state_bytes(None) == 0
    assert lib.ansatz_apply(None, None, None) == -1
    assert lib.energy(None, None, None) == -1
    assert lib.energy_grad(None, None, None, None, None, None) == -1
    assert lib.rdm1(None, None, None) == -1
    assert lib.set_onebody_potential(None, None) == -1


def test_batch_rejects_before_device(lib):
    # validation runs before any device call: empty batch, single precision,
    # an instance above the batch size limit, and a bad instance among good ones
    out = ctypes.c_void_p()
    assert lib.fsv_batch_create(ctypes.byref(out), None, 0, None) == -1
    cp, keep = _problem(precision=1)
    assert lib.fsv_batch_create(ctypes.byref(out), ctypes.byref(cp), 1, None) == -1
    assert b"FP64" in lib.fsv_last_error()
    cp, keep = _problem(n=26, na=3, nb=3)
    assert lib.fsv_batch_create(ctypes.byref(out), ctypes.byref(cp), 1, None) == -1
    assert b"24 qubits" in lib.fsv_last_error()
    from paper_2405_11567_amd import _lib
    good, k1 = _problem()
    bad, k2 = _problem(ops=[[0, 2, 1, 3]])
    arr = (_lib.Problem * 2)(good, bad)
    assert lib.fsv_batch_create(ctypes.byref(out), arr, 2, None) == -1
    assert b"instance 1" in lib.fsv_last_error()
    assert out.value is None
