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
