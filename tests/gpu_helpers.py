"""Shared helpers for the GPU tests: oracle results on the same seeded inputs."""

import numpy as np

from oracle import sector


def dense_from_sector(vec, p):
    idx = sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, p.ordering).astype(np.int64)
    out = np.zeros(1 << p.n_qubits, dtype=np.complex128)
    out[idx] = vec
    return out, idx


def oracle_state(p, theta=None):
    th = p.theta if theta is None else theta
    return sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, th, p.ordering)


def oracle_energy_grad(p, theta=None, h=None):
    th = p.theta if theta is None else theta
    hh = p.h if h is None else h
    return sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, th, hh, p.g, p.e_core, p.ordering)


def say(*a):
    print(*a, flush=True)


def random_dets(p, n_det, seed):
    """n_det distinct sector determinants of problem p (qubit strings in its
    ordering; the reference first) with random real coefficients, normalised."""
    idx = sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, p.ordering).astype(np.int64)
    rng = np.random.default_rng(seed)
    n_det = min(n_det, idx.size)
    pick = np.r_[0, 1 + rng.choice(idx.size - 1, n_det - 1, replace=False)]
    coef = rng.normal(size=n_det)
    coef[0] += 4.0
    return idx[pick].astype(np.uint64), coef / np.linalg.norm(coef)
