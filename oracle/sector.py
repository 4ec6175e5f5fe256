"""T3: ctypes wrapper over the sector-compressed C oracle (test infrastructure
only).  See sector.c for the definitions it follows.

Sector vectors are complex128 arrays of length C(M, N_alpha) * C(M, N_beta);
element r = Ia * nsb + Ib holds the amplitude of the qubit string
``sector_qubit_index(...)[r]`` of the dense state in the given ordering.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sector.c")
_LIB = os.path.join(_HERE, "liboracle_sector.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile sector.c with gcc -O2 -fopenmp into oracle/liboracle_sector.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        u64 = ctypes.POINTER(ctypes.c_uint64)
        c_int = ctypes.c_int
        lib.or_dim.restype = ctypes.c_long
        lib.or_dim.argtypes = [c_int, c_int, c_int]
        lib.or_sector_qubit_index.argtypes = [c_int, c_int, c_int, c_int, u64]
        lib.or_ansatz.argtypes = [c_int, c_int, c_int, c_int, c_int, i32, d, c_int, d]
        lib.or_apply_rotations.argtypes = [c_int, c_int, c_int, c_int, c_int, i32, d, c_int, d]
        lib.or_sigma.argtypes = [c_int, c_int, c_int, c_int, d, d, ctypes.c_double, d, d]
        lib.or_rdm1.argtypes = [c_int, c_int, c_int, c_int, d, d]
        lib.or_energy_grad.argtypes = [c_int, c_int, c_int, c_int, d, d, ctypes.c_double,
                                       c_int, i32, d, c_int, d, c_int, d, d]
        lib.or_pool_gradients.argtypes = [c_int, c_int, c_int, c_int, d, d, ctypes.c_double, d,
                                          c_int, i32, c_int, d]
        lib.or_num_threads.restype = c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().or_num_threads())


def dim(n_orb, n_alpha, n_beta) -> int:
    return comb(n_orb, n_alpha) * comb(n_orb, n_beta)


def sector_qubit_index(n_orb, n_alpha, n_beta, ordering=0) -> np.ndarray:
    out = np.zeros(dim(n_orb, n_alpha, n_beta), dtype=np.uint64)
    _check(_load().or_sector_qubit_index(n_orb, n_alpha, n_beta, ordering,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
           "sector_qubit_index")
    return out


def _ops(ops):
    return np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, 4))


def determinants_vector(n_orb, n_alpha, n_beta, dets, coef, ordering=0) -> np.ndarray:
    """Sector vector of sum_i coef_i |dets_i> for qubit strings dets (bit j =
    qubit j in the ordering); every determinant must lie in the sector."""
    idx = sector_qubit_index(n_orb, n_alpha, n_beta, ordering)
    pos = {int(x): r for r, x in enumerate(idx)}
    out = np.zeros(idx.size, dtype=np.complex128)
    for x, c in zip(dets, coef):
        out[pos[int(x)]] += c
    return out


def ansatz(n_orb, n_alpha, n_beta, ops, theta, ordering=0, excitation=0) -> np.ndarray:
    """Sector vector of U_K ... U_1 |ref> (excitation 0 fermionic, 1 qubit)."""
    ops = _ops(ops)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    psi = np.zeros(dim(n_orb, n_alpha, n_beta), dtype=np.complex128)
    _check(_load().or_ansatz(n_orb, n_alpha, n_beta, ordering, len(ops), _ip(ops), _dp(theta),
                             int(excitation), _dp(psi.view(np.float64))), "ansatz")
    return psi


def apply_rotations(psi, n_orb, n_alpha, n_beta, ops, theta, ordering=0, excitation=0) -> np.ndarray:
    ops = _ops(ops)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _check(_load().or_apply_rotations(n_orb, n_alpha, n_beta, ordering, len(ops), _ip(ops),
                                      _dp(theta), int(excitation), _dp(psi.view(np.float64))),
           "apply_rotations")
    return psi


def sigma(psi, h, g, e_core, n_alpha, n_beta, ordering=0) -> np.ndarray:
    """H psi on the sector (H as in sector.c; h already holds h + v)."""
    m = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    _check(_load().or_sigma(m, n_alpha, n_beta, ordering, _dp(h), _dp(g), float(e_core),
                            _dp(psi.view(np.float64)), _dp(out.view(np.float64))), "sigma")
    return out


def energy(psi, h, g, e_core, n_alpha, n_beta, ordering=0) -> float:
    return float(np.real(np.vdot(psi, sigma(psi, h, g, e_core, n_alpha, n_beta, ordering))))


def rdm1(psi, n_orb, n_alpha, n_beta, ordering=0) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    gam = np.zeros((2, n_orb, n_orb), dtype=np.complex128)
    _check(_load().or_rdm1(n_orb, n_alpha, n_beta, ordering, _dp(psi.view(np.float64)),
                           _dp(gam.view(np.float64))), "rdm1")
    return gam


def energy_grad(n_orb, n_alpha, n_beta, ops, theta, h, g, e_core, ordering=0, stride=None,
                excitation=0, psi0=None):
    """Stored-state adjoint: the state before every `stride`-th operator is
    kept and each segment is recomputed once (default: all states when they fit
    in 4 GiB, else stride ~ sqrt(K)).  psi0: initial sector vector (default
    the reference determinant)."""
    ops = _ops(ops)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    k = len(ops)
    if stride is None:
        vb = 16 * dim(n_orb, n_alpha, n_beta)
        stride = 1
        if (k + 2) * vb > (4 << 30):
            stride = max(1, int(np.ceil(np.sqrt(k))))
    e = ctypes.c_double(0.0)
    grad = np.zeros(k, dtype=np.float64)
    p0 = None
    if psi0 is not None:
        p0 = np.ascontiguousarray(psi0, dtype=np.complex128)
        if p0.size != dim(n_orb, n_alpha, n_beta):
            raise ValueError("psi0 must be a sector vector")
    _check(_load().or_energy_grad(n_orb, n_alpha, n_beta, ordering, _dp(h), _dp(g), float(e_core),
                                  k, _ip(ops), _dp(theta), int(excitation),
                                  _dp(p0.view(np.float64)) if p0 is not None else None, int(stride),
                                  ctypes.byref(e), _dp(grad)),
           "energy_grad")
    return float(e.value), grad


def pool_gradients(psi, h, g, e_core, pool, n_alpha, n_beta, ordering=0, excitation=0) -> np.ndarray:
    """ADAPT screening at the sector state psi: 2 Re <H psi| T_op |psi> for every
    pool operator (see sector.c)."""
    m = h.shape[0]
    pool = _ops(pool)
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros(len(pool), dtype=np.float64)
    _check(_load().or_pool_gradients(m, n_alpha, n_beta, ordering, _dp(h), _dp(g), float(e_core),
                                     _dp(psi.view(np.float64)), len(pool), _ip(pool), int(excitation),
                                     _dp(out)), "pool_gradients")
    return out


def fci_energy(h, g, e_core, n_alpha, n_beta, ordering=0, k=1) -> float:
    """Lowest sector eigenvalue by ARPACK Lanczos over the sector sigma."""
    import scipy.sparse.linalg as sla
    m = h.shape[0]
    n = dim(m, n_alpha, n_beta)
    if n <= 400:
        H = np.zeros((n, n), dtype=np.complex128)
        for i in range(n):
            e = np.zeros(n, dtype=np.complex128); e[i] = 1.0
            H[:, i] = sigma(e, h, g, e_core, n_alpha, n_beta, ordering)
        return float(np.linalg.eigvalsh(H)[0])
    op = sla.LinearOperator((n, n), dtype=np.complex128,
                            matvec=lambda v: sigma(v, h, g, e_core, n_alpha, n_beta, ordering))
    vals = sla.eigsh(op, k=k, which="SA", tol=1e-12)[0]
    return float(np.min(vals))
