"""T1: literal dense-state oracle (test infrastructure only).

The state is a 2^n complex128 vector; bit j of the basis index x is the
occupation of qubit j (one spin-orbital per qubit, Introduction).  Basis state
|x> = prod_{j ascending} (a^+_j)^{x_j} |vac>, so

    a_j |x>   = (-1)^popcount(x & (2^j - 1)) |x ^ 2^j>   if bit j of x is set,
    a^+_j |x> = (-1)^popcount(x & (2^j - 1)) |x ^ 2^j>   if bit j is clear,

and zero otherwise (Jordan-Wigner mapping, Strategy 2 density-matrix
paragraph).  Every operator below is applied one factor at a time, vectorised
over all basis states.

Spin-orbital label so = 2p + s (s = 0 alpha, 1 beta); the qubit holding it is
so for ordering 0 (interleaved) and p + s*M for ordering 1 (blocked).

Excitation kinds: 0 fermionic (the factors above, with their JW signs);
1 qubit excitation (the QEB operators of the paper's ADAPT pool, Computational
Details): the same factor list applied with qubit raising / lowering
operators, which flip the bit without any parity sign.
"""

from __future__ import annotations

import numpy as np


def qubit_of(so: int, n_orb: int, ordering: int) -> int:
    p, s = divmod(int(so), 2)
    return int(so) if ordering == 0 else p + s * n_orb


def apply_string(x: np.ndarray, factors, excitation: int = 0):
    """Apply operator factors (dagger, qubit) in the listed order (the first
    listed acts first) to every basis index in x.  Returns (x', sign, ok).
    excitation 1: qubit raising / lowering operators (no parity sign)."""
    x = x.copy()
    sign = np.ones(x.shape, dtype=np.int64)
    ok = np.ones(x.shape, dtype=bool)
    for dag, q in factors:
        bit = np.int64(1) << np.int64(q)
        occ = (x & bit) != 0
        ok &= (~occ) if dag else occ
        if excitation == 0:
            par = np.bitwise_count(x & (bit - 1)) & 1
            sign *= 1 - 2 * par.astype(np.int64)
        x ^= bit
    return x, sign, ok


def tau_factors(op, n_orb: int, ordering: int, adjoint: bool = False):
    """tau = a^+_a a^+_b a_j a_i for op = (a, b, j, i) (singles a^+_a a_i),
    listed in the order the factors act; adjoint gives tau^+."""
    a, b, j, i = (int(v) for v in op)
    q = lambda so: qubit_of(so, n_orb, ordering)  # noqa: E731
    if not adjoint:
        f = [(0, q(i))]
        if j >= 0:
            f.append((0, q(j)))
        if b >= 0:
            f.append((1, q(b)))
        f.append((1, q(a)))
    else:
        f = [(0, q(a))]
        if b >= 0:
            f.append((0, q(b)))
        if j >= 0:
            f.append((1, q(j)))
        f.append((1, q(i)))
    return f


def apply_operator(psi: np.ndarray, factors, coeff=1.0, excitation: int = 0) -> np.ndarray:
    """coeff * (operator string) psi as a new vector."""
    x = np.arange(psi.size, dtype=np.int64)
    xp, s, ok = apply_string(x, factors, excitation)
    out = np.zeros_like(psi)
    out[xp[ok]] = coeff * s[ok] * psi[x[ok]]
    return out


def reference_state(n_qubits: int, n_alpha: int, n_beta: int, ordering: int) -> np.ndarray:
    """Reference determinant: lowest n_alpha alpha and n_beta beta orbitals,
    amplitude +1 (the paper's HF initial state, Computational Details)."""
    m = n_qubits // 2
    x = 0
    for p in range(n_alpha):
        x |= 1 << qubit_of(2 * p, m, ordering)
    for p in range(n_beta):
        x |= 1 << qubit_of(2 * p + 1, m, ordering)
    psi = np.zeros(1 << n_qubits, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def rotate(psi: np.ndarray, op, theta: float, n_orb: int, ordering: int, excitation: int = 0) -> np.ndarray:
    """exp(theta (tau - tau^+)) psi.  On each pair tau|x> = s|x'>:
    psi'_x = cos psi_x - s sin psi_x',  psi'_x' = cos psi_x' + s sin psi_x."""
    psi = psi.copy()
    x = np.arange(psi.size, dtype=np.int64)
    xp, s, ok = apply_string(x, tau_factors(op, n_orb, ordering), excitation)
    src, dst, sg = x[ok], xp[ok], s[ok]
    a, b = psi[src].copy(), psi[dst].copy()
    c, sn = np.cos(theta), np.sin(theta)
    psi[src] = c * a - sg * sn * b
    psi[dst] = c * b + sg * sn * a
    return psi


def apply_T(psi: np.ndarray, op, n_orb: int, ordering: int, excitation: int = 0) -> np.ndarray:
    """(tau - tau^+) psi, both terms applied as operator strings."""
    return (apply_operator(psi, tau_factors(op, n_orb, ordering), excitation=excitation)
            - apply_operator(psi, tau_factors(op, n_orb, ordering, adjoint=True), excitation=excitation))


def ansatz_state(n_qubits, n_alpha, n_beta, ops, theta, ordering=0, excitation=0):
    """|psi(theta)> = U_K ... U_1 |ref>, first listed operator first."""
    m = n_qubits // 2
    psi = reference_state(n_qubits, n_alpha, n_beta, ordering)
    for op, t in zip(ops, theta):
        psi = rotate(psi, op, float(t), m, ordering, excitation)
    return psi


def hamiltonian_apply(psi, h, g, e_core, ordering=0):
    """H psi with H = E_core + sum_{pq,s} h_pq a^+_{ps} a_{qs}
    + 1/2 sum_{pqrs,st} (pq|rs) a^+_{ps} a^+_{rt} a_{st} a_{qs}
    (spatial chemist-notation integrals exchanged by FCIDUMP, Computational
    Details; the Strategy-2 potential enters by adding it to h, effective
    Hamiltonian equation).  Every term is applied literally."""
    m = h.shape[0]
    q = lambda p, s: qubit_of(2 * p + s, m, ordering)  # noqa: E731
    out = e_core * psi
    for s in (0, 1):
        for p in range(m):
            for qq in range(m):
                if h[p, qq] != 0.0:
                    out = out + apply_operator(psi, [(0, q(qq, s)), (1, q(p, s))], h[p, qq])
    for s in (0, 1):
        for t in (0, 1):
            for p in range(m):
                for qq in range(m):
                    for r in range(m):
                        for ss in range(m):
                            v = g[p, qq, r, ss]
                            if v == 0.0:
                                continue
                            f = [(0, q(qq, s)), (0, q(ss, t)), (1, q(r, t)), (1, q(p, s))]
                            out = out + apply_operator(psi, f, 0.5 * v)
    return out


def hamiltonian_apply_at(psi, xs, h, g, e_core, ordering=0) -> np.ndarray:
    """(H psi)[x] for the basis indices in xs only, every term of the same
    Hamiltonian as hamiltonian_apply applied literally: for a term c F,
    <x|F|y> is the sign of F^+ |x> = sign |y>, so (c F psi)[x] = c sign
    psi[y].  F^+ is the factor list reversed with creators and annihilators
    exchanged.  Costs O(#terms x len(xs)), so large states can be checked at
    sampled outputs."""
    m = h.shape[0]
    q = lambda p, s: qubit_of(2 * p + s, m, ordering)  # noqa: E731
    xs = np.asarray(xs, dtype=np.int64)
    out = e_core * psi[xs].astype(np.complex128)

    def add(factors, c):
        adj = [(1 - d, qq) for d, qq in reversed(factors)]
        y, sg, ok = apply_string(xs, adj)
        out[ok] += c * sg[ok] * psi[y[ok]]

    for s in (0, 1):
        for p in range(m):
            for qq in range(m):
                if h[p, qq] != 0.0:
                    add([(0, q(qq, s)), (1, q(p, s))], h[p, qq])
    for s in (0, 1):
        for t in (0, 1):
            for p in range(m):
                for qq in range(m):
                    for r in range(m):
                        for ss in range(m):
                            v = g[p, qq, r, ss]
                            if v != 0.0:
                                add([(0, q(qq, s)), (0, q(ss, t)), (1, q(r, t)), (1, q(p, s))], 0.5 * v)
    return out


def energy(psi, h, g, e_core, ordering=0) -> float:
    """E = Re <psi|H|psi> (the expectation value of Fig. 1), not normalised."""
    return float(np.real(np.vdot(psi, hamiltonian_apply(psi, h, g, e_core, ordering))))


def rdm1(psi, n_orb: int, ordering=0) -> np.ndarray:
    """gamma[s, p, q] = <psi| a^+_{ps} a_{qs} |psi> (Strategy 2, density-matrix
    equation), complex (2, M, M)."""
    gam = np.zeros((2, n_orb, n_orb), dtype=np.complex128)
    for s in (0, 1):
        for p in range(n_orb):
            for qq in range(n_orb):
                f = [(0, qubit_of(2 * qq + s, n_orb, ordering)), (1, qubit_of(2 * p + s, n_orb, ordering))]
                gam[s, p, qq] = np.vdot(psi, apply_operator(psi, f))
    return gam


def energy_grad(n_qubits, n_alpha, n_beta, ops, theta, h, g, e_core, ordering=0, excitation=0):
    """Energy and dE/dtheta_k = 2 Re <lam_k| T_k |psi_k>, with every forward
    state psi_k stored and lam_k = U_{k+1}^+ ... U_K^+ H psi_K."""
    m = n_qubits // 2
    states = [reference_state(n_qubits, n_alpha, n_beta, ordering)]
    for op, t in zip(ops, theta):
        states.append(rotate(states[-1], op, float(t), m, ordering, excitation))
    lam = hamiltonian_apply(states[-1], h, g, e_core, ordering)
    e = float(np.real(np.vdot(states[-1], lam)))
    grad = np.zeros(len(ops))
    for k in range(len(ops) - 1, -1, -1):
        grad[k] = 2.0 * np.real(np.vdot(lam, apply_T(states[k + 1], ops[k], m, ordering, excitation)))
        lam = rotate(lam, ops[k], -float(theta[k]), m, ordering, excitation)
    return e, grad


def energy_fd_grad(n_qubits, n_alpha, n_beta, ops, theta, h, g, e_core, ordering=0, step=1e-5,
                   excitation=0):
    """Central finite differences of the energy, step h = 1e-5."""
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.zeros(len(theta))
    for k in range(len(theta)):
        tp = theta.copy(); tp[k] += step
        tm = theta.copy(); tm[k] -= step
        ep = energy(ansatz_state(n_qubits, n_alpha, n_beta, ops, tp, ordering, excitation), h, g, e_core, ordering)
        em = energy(ansatz_state(n_qubits, n_alpha, n_beta, ops, tm, ordering, excitation), h, g, e_core, ordering)
        grad[k] = (ep - em) / (2 * step)
    return grad


def pool_gradients(psi, h, g, e_core, pool, n_orb, ordering=0, excitation=0):
    """ADAPT screening of an operator pool at the state psi: for every pool
    operator, the derivative of the energy with respect to its angle when it
    is appended to the ansatz at angle 0,
        g_op = <psi| [H, T_op] |psi> = 2 Re <H psi| T_op |psi>
    (real H, anti-Hermitian T_op)."""
    lam = hamiltonian_apply(psi, h, g, e_core, ordering)
    return np.array([2.0 * np.real(np.vdot(lam, apply_T(psi, op, n_orb, ordering, excitation))) for op in pool])
