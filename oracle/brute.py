"""T2: brute-force matrix oracle (test infrastructure only).

Every fermionic operator is a 2^n x 2^n sparse matrix built from Kronecker
products of Jordan-Wigner factors: a_j = I x ... x I x sigma^- x Z x ... x Z,
with Z on every qubit below j (bit j of the basis index is qubit j, so the
rightmost Kronecker factor acts on qubit 0).  Rotations are matrix
exponentials exp(theta T) of T = tau - tau^+ (for qubit excitations the
same products with the Z strings left out), and the FCI energy (the
finite-basis minimum of the energy functional, Density-based basis-set
correction section) is the lowest eigenvalue of H restricted to the
(N_alpha, N_beta) sector.  Independent of the bit-manipulation route of T1/T3.
Practical for n <= 10.
"""

from __future__ import annotations

from functools import lru_cache

import numpy as np
import scipy.linalg
import scipy.sparse as sp

_I = sp.identity(2, format="csr", dtype=np.complex128)
_Z = sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=np.complex128))
_LOWER = sp.csr_matrix(np.array([[0, 1], [0, 0]], dtype=np.complex128))  # |0><1|


@lru_cache(maxsize=64)
def annihilator(j: int, n: int) -> sp.csr_matrix:
    mat = sp.identity(1, format="csr", dtype=np.complex128)
    for qubit in range(n - 1, -1, -1):  # leftmost factor = highest qubit
        if qubit > j:
            f = _I
        elif qubit == j:
            f = _LOWER
        else:
            f = _Z
        mat = sp.kron(mat, f, format="csr")
    return mat


def creator(j: int, n: int) -> sp.csr_matrix:
    return annihilator(j, n).conj().T.tocsr()


@lru_cache(maxsize=64)
def qubit_lowering(j: int, n: int) -> sp.csr_matrix:
    """|0><1| on qubit j, identity elsewhere (no Z string)."""
    mat = sp.identity(1, format="csr", dtype=np.complex128)
    for qubit in range(n - 1, -1, -1):
        mat = sp.kron(mat, _LOWER if qubit == j else _I, format="csr")
    return mat


def qubit_raising(j: int, n: int) -> sp.csr_matrix:
    return qubit_lowering(j, n).conj().T.tocsr()


def _q(so, m, ordering):
    p, s = divmod(int(so), 2)
    return int(so) if ordering == 0 else p + s * m


def tau_matrix(op, n: int, ordering: int, excitation: int = 0) -> sp.csr_matrix:
    """tau = a^+_a a^+_b a_j a_i (excitation 0) or Q^+_a Q^+_b Q_j Q_i with
    qubit raising / lowering operators (excitation 1)."""
    a, b, j, i = (int(v) for v in op)
    m = n // 2
    up, down = (creator, annihilator) if excitation == 0 else (qubit_raising, qubit_lowering)
    if b < 0:
        return (up(_q(a, m, ordering), n) @ down(_q(i, m, ordering), n)).tocsr()
    return (up(_q(a, m, ordering), n) @ up(_q(b, m, ordering), n)
            @ down(_q(j, m, ordering), n) @ down(_q(i, m, ordering), n)).tocsr()


def hamiltonian_matrix(h, g, e_core, n: int, ordering: int) -> sp.csr_matrix:
    m = n // 2
    dim = 1 << n
    H = e_core * sp.identity(dim, format="csr", dtype=np.complex128)
    A = {(p, s): annihilator(_q(2 * p + s, m, ordering), n) for p in range(m) for s in (0, 1)}
    C = {k: v.conj().T.tocsr() for k, v in A.items()}
    for s in (0, 1):
        for p in range(m):
            for q in range(m):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * (C[p, s] @ A[q, s])
    for s in (0, 1):
        for t in (0, 1):
            for p in range(m):
                for q in range(m):
                    for r in range(m):
                        for u in range(m):
                            v = g[p, q, r, u]
                            if v != 0.0:
                                H = H + 0.5 * v * (C[p, s] @ C[r, t] @ A[u, t] @ A[q, s])
    return H.tocsr()


def reference_index(n, n_alpha, n_beta, ordering) -> int:
    m = n // 2
    x = 0
    for p in range(n_alpha):
        x |= 1 << _q(2 * p, m, ordering)
    for p in range(n_beta):
        x |= 1 << _q(2 * p + 1, m, ordering)
    return x


def ansatz_state(n, n_alpha, n_beta, ops, theta, ordering=0, excitation=0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[reference_index(n, n_alpha, n_beta, ordering)] = 1.0
    for op, t in zip(ops, theta):
        tau = tau_matrix(op, n, ordering, excitation).toarray()
        U = scipy.linalg.expm(float(t) * (tau - tau.conj().T))
        psi = U @ psi
    return psi


def sector_indices(n, n_alpha, n_beta, ordering) -> np.ndarray:
    m = n // 2
    x = np.arange(1 << n, dtype=np.int64)
    na = np.zeros_like(x)
    nb = np.zeros_like(x)
    for p in range(m):
        na += (x >> _q(2 * p, m, ordering)) & 1
        nb += (x >> _q(2 * p + 1, m, ordering)) & 1
    return np.nonzero((na == n_alpha) & (nb == n_beta))[0]


def fci_energy(h, g, e_core, n, n_alpha, n_beta, ordering=0) -> float:
    H = hamiltonian_matrix(h, g, e_core, n, ordering)
    idx = sector_indices(n, n_alpha, n_beta, ordering)
    Hs = H[idx][:, idx].toarray()
    return float(np.linalg.eigvalsh(Hs)[0])
