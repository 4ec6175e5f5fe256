"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper's molecules (H2O, N2, LiH, H2 and hydrogen chains at 4-32 qubits,
Tables II and IV) are represented only by their shapes: qubit counts, electron
counts and ansatz sizes that are mostly double excitations.  Their integrals
are not available, so a synthetic Hamiltonian with the same structure stands in
for them:

* h: real symmetric M x M, diagonal evenly spaced from -1.0 to +0.5,
  off-diagonal upper triangle i.i.d. N(0, 0.1), mirrored;
* g: chemist-notation (pq|rs) = sum_l L_l[p,q] L_l[r,s] with 8 real symmetric
  factors L_l whose upper triangles (diagonal included) are i.i.d. N(0, 0.05).
  This makes g 8-fold symmetric and positive semidefinite as a supermatrix.

Draw order inside one generator: h off-diagonal (row-major upper triangle),
then L_0..L_7 (row-major upper triangle with diagonal), then the operator
indices, then the angles.  Generator: numpy PCG64 via default_rng(seed).

Spin-orbital labels are canonical: so = 2*p + sigma (sigma 0 = alpha, 1 = beta),
independent of the qubit ordering a plan uses in memory.  An operator is the
tuple (a, b, j, i) meaning a^+_a a^+_b a_j a_i; a single excitation is
(a, -1, -1, i) meaning a^+_a a_i.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")
N_FACTORS = 8


@dataclass
class Problem:
    n_qubits: int
    n_alpha: int
    n_beta: int
    h: np.ndarray                 # (M, M) float64
    g: np.ndarray                 # (M, M, M, M) float64, chemist (pq|rs)
    ops: np.ndarray               # (K, 4) int32, (a, b, j, i)
    theta: np.ndarray             # (K,) float64
    e_core: float = 0.0
    ordering: int = 0             # 0 interleaved (qubit 2p+s), 1 blocked (p + s*M)
    name: str = ""
    meta: dict = field(default_factory=dict)
    excitation: int = 0           # 0 fermionic excitations, 1 qubit excitations

    @property
    def n_orb(self) -> int:
        return self.n_qubits // 2

    @property
    def n_ops(self) -> int:
        return int(self.ops.shape[0])

    def with_ordering(self, ordering: int) -> "Problem":
        return Problem(self.n_qubits, self.n_alpha, self.n_beta, self.h, self.g,
                       self.ops, self.theta, self.e_core, ordering, self.name,
                       dict(self.meta))


def _sym_upper(rng: np.random.Generator, m: int, std: float, diag: bool) -> np.ndarray:
    """Symmetric matrix from i.i.d. normal upper-triangle draws (row-major)."""
    a = np.zeros((m, m))
    k = 0 if diag else 1
    iu = np.triu_indices(m, k=k)
    a[iu] = rng.normal(0.0, std, size=len(iu[0]))
    a = a + np.triu(a, 1).T
    return a


def synthetic_hamiltonian(m: int, rng: np.random.Generator):
    h = _sym_upper(rng, m, 0.1, diag=False)
    h[np.diag_indices(m)] = np.linspace(-1.0, 0.5, m)
    g = np.zeros((m, m, m, m))
    for _ in range(N_FACTORS):
        l = _sym_upper(rng, m, 0.05, diag=True)
        g += np.einsum("pq,rs->pqrs", l, l)
    return h, g


def uccsd_pool(m: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """All spin-conserving occupied->virtual singles and doubles relative to the
    reference determinant that fills the lowest n_alpha alpha and n_beta beta
    orbitals.  Canonical order: singles alpha, singles beta, doubles aa, bb, ab,
    each lexicographic in (i, j, a, b)."""
    occ = [list(range(n_alpha)), list(range(n_beta))]
    vir = [list(range(n_alpha, m)), list(range(n_beta, m))]
    so = lambda p, s: 2 * p + s  # noqa: E731
    pool = []
    for s in (0, 1):
        for i in occ[s]:
            for a in vir[s]:
                pool.append((so(a, s), -1, -1, so(i, s)))
    for s in (0, 1):
        for i in occ[s]:
            for j in occ[s]:
                if j <= i:
                    continue
                for a in vir[s]:
                    for b in vir[s]:
                        if b <= a:
                            continue
                        pool.append((so(a, s), so(b, s), so(j, s), so(i, s)))
    for i in occ[0]:
        for j in occ[1]:
            for a in vir[0]:
                for b in vir[1]:
                    pool.append((so(a, 0), so(b, 1), so(j, 1), so(i, 0)))
    return np.asarray(pool, dtype=np.int32).reshape(-1, 4)


def random_problem(n_qubits: int, n_electrons: int, n_ops: Optional[int], seed: int,
                   theta_std: float = 0.1, replace: bool = False,
                   ordering: int = 0, name: str = "") -> Problem:
    """One seeded instance.  n_ops=None takes the whole pool in canonical order."""
    m = n_qubits // 2
    na = (n_electrons + 1) // 2
    nb = n_electrons // 2
    rng = np.random.default_rng(seed)
    h, g = synthetic_hamiltonian(m, rng)
    pool = uccsd_pool(m, na, nb)
    if n_ops is None:
        ops = pool.copy()
    else:
        if replace:
            idx = rng.integers(0, len(pool), size=n_ops)
        else:
            idx = rng.choice(len(pool), size=n_ops, replace=False)
        ops = pool[idx]
    theta = rng.normal(0.0, theta_std, size=len(ops))
    return Problem(n_qubits, na, nb, h, g, np.ascontiguousarray(ops, dtype=np.int32),
                   theta.astype(np.float64), 0.0, ordering, name,
                   {"seed": seed, "pool_size": len(pool)})


def config(name: str, ordering: int = 0) -> Problem:
    """The five workload shapes: C1 8 qubits / 4 electrons / all 26 UCCSD ops;
    C2 16 / 8 / all 360; C3 24 / 12 / 200 sampled of 1818; C5 30 / 14 / 500
    sampled of 4424.  C4 is the batch (see batch_config)."""
    if name == "C1":
        return random_problem(8, 4, None, seed=1, theta_std=0.05, ordering=ordering, name=name)
    if name == "C2":
        return random_problem(16, 8, None, seed=2, theta_std=0.05, ordering=ordering, name=name)
    if name == "C3":
        return random_problem(24, 12, 200, seed=3, theta_std=0.1, ordering=ordering, name=name)
    if name == "C5":
        return random_problem(30, 14, 500, seed=5, theta_std=0.05, ordering=ordering, name=name)
    raise ValueError(f"unknown config {name!r}")


def batch_config(count: int = 256, ordering: int = 0) -> List[Problem]:
    """C4: independent instances with qubit counts uniform over the even values
    10..20, electrons = qubits/2 + U{-2..2}, 50..150 operators sampled with
    replacement, theta ~ N(0, 0.1).  Shapes come from seed 4, instance i from
    seed 4000 + i."""
    shape_rng = np.random.default_rng(4)
    out = []
    for i in range(count):
        n = int(shape_rng.choice(np.arange(10, 21, 2)))
        ne = n // 2 + int(shape_rng.integers(-2, 3))
        k = int(shape_rng.integers(50, 151))
        out.append(random_problem(n, ne, k, seed=4000 + i, theta_std=0.1, replace=True,
                                  ordering=ordering, name=f"C4[{i}]"))
    return out


def potential_v0(m: int, seed: int = 33, std: float = 0.02) -> np.ndarray:
    """Symmetric one-body potential with N(0, std) upper triangle (diagonal
    included), the stand-in for the basis-set correction potential."""
    rng = np.random.default_rng(seed)
    return _sym_upper(rng, m, std, diag=True)
