"""Pins of the oracle's qubit-excitation (QEB) operators, ADAPT pool screening,
multi-determinant initial states and one-body properties
against brute force, finite differences and exact relations.

ADAPT screening value of a pool operator T at a state psi: the derivative of
the energy when U = exp(theta T) is appended to the ansatz, at theta = 0,
    g = d/dtheta <psi| U^+ H U |psi> = <psi| [H, T] |psi> = 2 Re <H psi| T |psi>.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import brute, dense, sector
from workloads import random_problem, uccsd_pool


def _idx(p):
    return sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, p.ordering).astype(np.int64)


# --------------------------------------------------------------- P9 ----------
@pytest.mark.parametrize("ordering", [0, 1])
def test_qubit_excitations_brute_force(ordering):
    # QEB rotations: Kronecker products of qubit raising / lowering matrices
    # and expm (T2) against the bit-flip routes of T1 and T3
    p = random_problem(8, 4, None, seed=61, theta_std=0.4, ordering=ordering)
    m = p.n_orb
    psi_b = brute.ansatz_state(8, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation=1)
    psi_d = dense.ansatz_state(8, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation=1)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation=1)
    assert np.abs(psi_b - psi_d).max() < 1e-13
    assert np.abs(psi_b[_idx(p)] - psi_s).max() < 1e-13
    assert abs(np.linalg.norm(psi_s) - 1.0) < 1e-13
    # a genuinely different operator family: the fermionic state differs
    psi_f = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation=0)
    assert np.abs(psi_f - psi_s).max() > 1e-3
    H = brute.hamiltonian_matrix(p.h, p.g, 0.0, 8, ordering)
    e_b = np.real(np.vdot(psi_b, H @ psi_b))
    assert abs(e_b - sector.energy(psi_s, p.h, p.g, 0.0, p.n_alpha, p.n_beta, ordering)) < 1e-12
    # U(-theta) U(theta) = 1 for every qubit excitation
    back = sector.apply_rotations(psi_s, m, p.n_alpha, p.n_beta, p.ops[::-1], -p.theta[::-1],
                                  ordering, excitation=1)
    ref = np.zeros_like(back)
    ref[0] = 1.0
    assert np.abs(back - ref).max() < 1e-13


# --------------------------------------------------------------- P10 ---------
@pytest.mark.parametrize("ordering", [0, 1])
def test_pool_at_reference_qeb_vs_fermionic(ordering):
    # At the reference determinant tau|ref> = s|x'> with s the JW sign of the
    # fermionic operator (+1 for the qubit operator), so the screening values
    # differ exactly by s; s is read off the brute-force fermionic matrix.
    n, ne = 10, 6
    p = random_problem(n, ne, None, seed=62, ordering=ordering)
    m = n // 2
    pool = p.ops
    psi = sector.ansatz(m, p.n_alpha, p.n_beta, pool[:0], np.zeros(0), ordering)
    g_f = sector.pool_gradients(psi, p.h, p.g, 0.0, pool, p.n_alpha, p.n_beta, ordering, 0)
    g_q = sector.pool_gradients(psi, p.h, p.g, 0.0, pool, p.n_alpha, p.n_beta, ordering, 1)
    x0 = brute.reference_index(n, p.n_alpha, p.n_beta, ordering)
    signs = []
    for op in pool:
        col = brute.tau_matrix(op, n, ordering).tocsc()[:, x0]
        nz = col.nonzero()[0]
        assert len(nz) == 1
        signs.append(np.real(col[nz[0], 0]))
    signs = np.array(signs)
    assert set(np.unique(signs)) <= {-1.0, 1.0}
    assert np.abs(g_q - signs * g_f).max() < 1e-13
    assert (signs < 0).any() and (signs > 0).any()  # both cases are exercised


# --------------------------------------------------------------- P11 ---------
@pytest.mark.parametrize("excitation", [0, 1])
@pytest.mark.parametrize("ordering", [0, 1])
def test_pool_gradients_finite_difference(excitation, ordering):
    # screening value = central difference of the energy with the pool
    # operator appended (T1, dense), and T1 = T3
    p = random_problem(8, 4, 10, seed=63, theta_std=0.4, ordering=ordering)
    m, n = p.n_orb, 8
    pool = np.asarray(uccsd_pool(m, p.n_alpha, p.n_beta), dtype=np.int32)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation)
    g3 = sector.pool_gradients(psi_s, p.h, p.g, 0.2, pool, p.n_alpha, p.n_beta, ordering, excitation)
    psi_d = dense.ansatz_state(n, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation)
    g1 = dense.pool_gradients(psi_d, p.h, p.g, 0.2, pool, m, ordering, excitation)
    assert np.abs(g1 - g3).max() < 1e-12
    h = 1e-5
    for t, op in enumerate(pool):
        ops = np.vstack([p.ops, op[None, :]])
        ep = dense.energy(dense.ansatz_state(n, p.n_alpha, p.n_beta, ops, np.r_[p.theta, h], ordering,
                                             excitation), p.h, p.g, 0.2, ordering)
        em = dense.energy(dense.ansatz_state(n, p.n_alpha, p.n_beta, ops, np.r_[p.theta, -h], ordering,
                                             excitation), p.h, p.g, 0.2, ordering)
        assert abs((ep - em) / (2 * h) - g3[t]) < 1e-8


# --------------------------------------------------------------- P12 ---------
@pytest.mark.parametrize("ordering", [0, 1])
def test_qubit_excitation_adjoint_gradient(ordering):
    # adjoint gradient of a QEB ansatz vs finite differences; the screening
    # value of the last ansatz operator at the final state equals its own
    # gradient (T_K commutes with U_K)
    p = random_problem(10, 5, 14, seed=64, theta_std=0.4, ordering=ordering)
    m = p.n_orb
    e, g = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, ordering,
                              excitation=1)
    gfd = dense.energy_fd_grad(10, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, ordering,
                               excitation=1)
    assert np.abs(g - gfd).max() < 1e-7
    psi = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation=1)
    last = sector.pool_gradients(psi, p.h, p.g, 0.0, p.ops[-1:], p.n_alpha, p.n_beta, ordering, 1)
    assert abs(last[0] - g[-1]) < 1e-12
    assert abs(sector.energy(psi, p.h, p.g, 0.0, p.n_alpha, p.n_beta, ordering) - e) < 1e-12


def test_qubit_single_without_crossing_equals_fermionic():
    # a single excitation between neighbouring qubits has no JW string, so the
    # qubit and fermionic rotations coincide on every state (blocked ordering:
    # alpha orbitals 2 -> 3 are qubits 2 and 3)
    p = random_problem(10, 5, 20, seed=65, theta_std=0.4, ordering=1)
    m = p.n_orb
    psi = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, 1)
    op = np.array([[6, -1, -1, 4]], dtype=np.int32)  # alpha 3 <- alpha 2
    a = sector.apply_rotations(psi, m, p.n_alpha, p.n_beta, op, [0.7], 1, excitation=0)
    b = sector.apply_rotations(psi, m, p.n_alpha, p.n_beta, op, [0.7], 1, excitation=1)
    assert np.abs(a - b).max() < 1e-15


# --------------------------------------------------------------- P13-P15 -----
def _random_dets(p, n_det, seed):
    """n_det distinct sector determinants (qubit strings) and normalised real
    coefficients, the reference first."""
    idx = sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, p.ordering).astype(np.int64)
    rng = np.random.default_rng(seed)
    pick = np.r_[0, 1 + rng.choice(idx.size - 1, n_det - 1, replace=False)]
    coef = rng.normal(size=n_det)
    coef[0] += 3.0
    return idx[pick], coef / np.linalg.norm(coef)


@pytest.mark.parametrize("ordering", [0, 1])
def test_multideterminant_start_brute_force(ordering):
    # a multi-determinant initial state: energy at theta = 0 is Phi^T H Phi
    # (brute-force matrix), and the rotations applied to it match expm products
    p = random_problem(8, 4, 12, seed=71, theta_std=0.4, ordering=ordering)
    m, n = p.n_orb, 8
    dets, coef = _random_dets(p, 6, 72)
    phi = np.zeros(1 << n, dtype=np.complex128)
    phi[dets] = coef
    H = brute.hamiltonian_matrix(p.h, p.g, 0.3, n, ordering)
    psi0 = sector.determinants_vector(m, p.n_alpha, p.n_beta, dets, coef, ordering)
    e0, _ = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops[:0], np.zeros(0), p.h, p.g, 0.3, ordering,
                               psi0=psi0)
    assert abs(e0 - np.real(np.vdot(phi, H @ phi))) < 1e-12
    psi_b = phi.copy()
    for op, t in zip(p.ops, p.theta):
        tau = brute.tau_matrix(op, n, ordering).toarray()
        psi_b = scipy.linalg.expm(float(t) * (tau - tau.conj().T)) @ psi_b
    psi_s = sector.apply_rotations(psi0, m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    assert np.abs(psi_b[_idx(p)] - psi_s).max() < 1e-13
    e, _ = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.3, ordering, psi0=psi0)
    assert abs(e - np.real(np.vdot(psi_b, H @ psi_b))) < 1e-12


def test_multideterminant_gradient_finite_difference():
    p = random_problem(10, 5, 15, seed=73, theta_std=0.4, ordering=0)
    m = p.n_orb
    dets, coef = _random_dets(p, 12, 74)
    psi0 = sector.determinants_vector(m, p.n_alpha, p.n_beta, dets, coef, 0)
    e, g = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, 0, psi0=psi0)
    h = 1e-5
    for k in range(p.n_ops):
        tp, tm = p.theta.copy(), p.theta.copy()
        tp[k] += h
        tm[k] -= h
        ep = sector.energy(sector.apply_rotations(psi0, m, p.n_alpha, p.n_beta, p.ops, tp, 0), p.h, p.g, 0.0,
                           p.n_alpha, p.n_beta, 0)
        em = sector.energy(sector.apply_rotations(psi0, m, p.n_alpha, p.n_beta, p.ops, tm, 0), p.h, p.g, 0.0,
                           p.n_alpha, p.n_beta, 0)
        assert abs((ep - em) / (2 * h) - g[k]) < 1e-8


@pytest.mark.parametrize("ordering", [0, 1])
def test_onebody_property_brute_force(ordering):
    # a first-order property <psi|D|psi>, D = sum_{pq,s} d_pq a^+_{ps} a_{qs}
    # (a dipole component for dipole integrals d), equals tr(d (gamma_a + gamma_b))
    p = random_problem(8, 3, 10, seed=75, theta_std=0.5, ordering=ordering)
    m, n = p.n_orb, 8
    rng = np.random.default_rng(76)
    d = rng.normal(size=(m, m))  # need not be symmetric
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    gam = sector.rdm1(psi_s, m, p.n_alpha, p.n_beta, ordering)
    val = np.sum(d * (gam[0] + gam[1]))
    D = sum(d[a, b] * (brute.creator(brute._q(2 * a + s, m, ordering), n)
                       @ brute.annihilator(brute._q(2 * b + s, m, ordering), n))
            for a in range(m) for b in range(m) for s in (0, 1))
    psi_b = brute.ansatz_state(n, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    assert abs(val - np.vdot(psi_b, D @ psi_b)) < 1e-12
