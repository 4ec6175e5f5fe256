"""Pins of the FP64 oracle against what the definitions and the mathematics fix
(closed forms, invariants, brute force), independent of the oracle's own code.

Each pin is chosen so that a plausible mistake (a dropped spin block, a wrong
JW sign, a transposed integral index, a missing 1/2) fails at least one test.
"""

import itertools

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import brute, dense, sector
from workloads import config, random_problem, uccsd_pool


def so_list(n_alpha, n_beta):
    return [(p, 0) for p in range(n_alpha)] + [(p, 1) for p in range(n_beta)]


def slater_condon_energy(h, g, e_core, occ):
    """Closed-form energy of one determinant with occupied (orbital, spin) set."""
    e = e_core + sum(h[p, p] for p, _ in occ)
    for (p, s), (q, t) in itertools.product(occ, occ):
        e += 0.5 * g[p, p, q, q]
        if s == t:
            e -= 0.5 * g[p, q, q, p]
    return e


# ---------------------------------------------------------------- P1 ---------
@pytest.mark.parametrize("n,ne,ordering", [(8, 4, 0), (8, 3, 1), (10, 6, 0), (12, 5, 1)])
def test_reference_energy_closed_form(n, ne, ordering):
    p = random_problem(n, ne, 3, seed=100 + n + ne, ordering=ordering)
    e_core = 0.37
    occ = so_list(p.n_alpha, p.n_beta)
    ref = slater_condon_energy(p.h, p.g, e_core, occ)
    psi = dense.reference_state(n, p.n_alpha, p.n_beta, ordering)
    assert abs(dense.energy(psi, p.h, p.g, e_core, ordering) - ref) < 1e-12
    m = n // 2
    s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, np.zeros(3), ordering)
    assert abs(sector.energy(s, p.h, p.g, e_core, p.n_alpha, p.n_beta, ordering) - ref) < 1e-12


# ---------------------------------------------------------------- P2 ---------
def fock_ai(h, g, occ, a, sa, i):
    v = h[a, i]
    for (j, t) in occ:
        v += g[a, i, j, j]
        if t == sa:
            v -= g[a, j, j, i]
    return v


@pytest.mark.parametrize("ordering", [0, 1])
def test_gradient_at_zero_closed_form(ordering):
    n, ne = 10, 6
    p = random_problem(n, ne, None, seed=7, ordering=ordering)
    m = n // 2
    occ = so_list(p.n_alpha, p.n_beta)
    e, grad = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, np.zeros(p.n_ops),
                                 p.h, p.g, 0.0, ordering)
    expect = np.zeros(p.n_ops)
    for k, (a, b, j, i) in enumerate(p.ops):
        if b < 0:
            expect[k] = 2 * fock_ai(p.h, p.g, occ, a // 2, a % 2, i // 2)
        else:
            A, B, J, I = a // 2, b // 2, j // 2, i // 2
            sA, sB, sJ, sI = a % 2, b % 2, j % 2, i % 2
            v = 0.0
            if sI == sA and sJ == sB:
                v += p.g[I, A, J, B]
            if sI == sB and sJ == sA:
                v -= p.g[I, B, J, A]
            expect[k] = 2 * v
    assert np.abs(grad - expect).max() < 1e-12
    assert abs(e - slater_condon_energy(p.h, p.g, 0.0, occ)) < 1e-12


# ---------------------------------------------------------------- P3 ---------
def test_one_rotation_closed_form():
    n, ne = 10, 4
    p = random_problem(n, ne, None, seed=21)
    m = n // 2
    occ = so_list(p.n_alpha, p.n_beta)
    e_hf = slater_condon_energy(p.h, p.g, 0.0, occ)
    doubles = [op for op in p.ops if op[1] >= 0]
    for op in doubles[:6]:
        a, b, j, i = (int(v) for v in op)
        occ_d = [o for o in occ if 2 * o[0] + o[1] not in (i, j)] + [(a // 2, a % 2), (b // 2, b % 2)]
        e_d = slater_condon_energy(p.h, p.g, 0.0, occ_d)
        _, g0 = sector.energy_grad(m, p.n_alpha, p.n_beta, [op], [0.0], p.h, p.g, 0.0)
        for th in (0.3, -1.1, np.pi / 2):
            psi = sector.ansatz(m, p.n_alpha, p.n_beta, [op], [th])
            e = sector.energy(psi, p.h, p.g, 0.0, p.n_alpha, p.n_beta)
            expect = np.cos(th) ** 2 * e_hf + np.sin(th) ** 2 * e_d + np.sin(2 * th) * g0[0] / 2
            assert abs(e - expect) < 1e-12


# ---------------------------------------------------------------- P4 ---------
@pytest.mark.parametrize("ordering", [0, 1])
def test_singles_thouless_closed_form(ordering):
    n, ne = 12, 5
    p = random_problem(n, ne, None, seed=31, ordering=ordering)
    m = n // 2
    rng = np.random.default_rng(5)
    singles = [op for op in p.ops if op[1] < 0]
    ops = [singles[i] for i in rng.integers(0, len(singles), 14)]
    theta = rng.normal(0, 0.4, len(ops))
    psi = sector.ansatz(m, p.n_alpha, p.n_beta, ops, theta, ordering)
    gam = sector.rdm1(psi, m, p.n_alpha, p.n_beta, ordering)
    for s, ne_s in ((0, p.n_alpha), (1, p.n_beta)):
        C = np.eye(m)
        for op, t in zip(ops, theta):
            a, i = op[0], op[3]
            if a % 2 != s:
                continue
            kap = np.zeros((m, m))
            kap[a // 2, i // 2] = t
            kap[i // 2, a // 2] = -t
            C = scipy.linalg.expm(kap) @ C
        Cocc = C[:, :ne_s]
        assert np.abs(gam[s] - Cocc @ Cocc.T).max() < 1e-12
    # with g = 0 the energy is the one-body trace
    g0 = np.zeros_like(p.g)
    e = sector.energy(psi, p.h, g0, 0.25, p.n_alpha, p.n_beta, ordering)
    assert abs(e - (0.25 + np.trace(p.h @ (gam[0] + gam[1]).real))) < 1e-12


# ---------------------------------------------------------------- P5 ---------
@pytest.mark.parametrize("ordering", [0, 1])
def test_brute_force_matches_dense_and_sector(ordering):
    p = random_problem(8, 4, None, seed=41, theta_std=0.4, ordering=ordering)
    m = p.n_orb
    psi_b = brute.ansatz_state(8, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    psi_d = dense.ansatz_state(8, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    idx = sector.sector_qubit_index(m, p.n_alpha, p.n_beta, ordering).astype(np.int64)
    assert np.abs(psi_b - psi_d).max() < 1e-13
    assert np.abs(psi_b[idx] - psi_s).max() < 1e-13
    H = brute.hamiltonian_matrix(p.h, p.g, 0.1, 8, ordering)
    assert abs(H - H.conj().T).max() < 1e-14
    e_b = np.real(np.vdot(psi_b, H @ psi_b))
    assert abs(e_b - sector.energy(psi_s, p.h, p.g, 0.1, p.n_alpha, p.n_beta, ordering)) < 1e-12
    sig_b = H @ psi_b
    sig_s = sector.sigma(psi_s, p.h, p.g, 0.1, p.n_alpha, p.n_beta, ordering)
    assert np.abs(sig_b[idx] - sig_s).max() < 1e-12


def test_brute_force_odd_electrons_blocked():
    p = random_problem(10, 5, 12, seed=43, theta_std=0.5, ordering=1)
    m = p.n_orb
    psi_b = brute.ansatz_state(10, p.n_alpha, p.n_beta, p.ops, p.theta, 1)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, 1)
    idx = sector.sector_qubit_index(m, p.n_alpha, p.n_beta, 1).astype(np.int64)
    assert np.abs(psi_b[idx] - psi_s).max() < 1e-13
    H = brute.hamiltonian_matrix(p.h, p.g, 0.0, 10, 1)
    sig_s = sector.sigma(psi_s, p.h, p.g, 0.0, p.n_alpha, p.n_beta, 1)
    assert np.abs((H @ psi_b)[idx] - sig_s).max() < 1e-12


# ---------------------------------------------------------------- T1 vs T3 ----
@pytest.mark.parametrize("n,ne,seed,ordering", [(10, 5, 51, 0), (12, 6, 52, 1), (12, 7, 53, 0)])
def test_dense_literal_matches_sector(n, ne, seed, ordering):
    p = random_problem(n, ne, 20, seed=seed, theta_std=0.4, ordering=ordering)
    m = p.n_orb
    psi_d = dense.ansatz_state(n, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    idx = sector.sector_qubit_index(m, p.n_alpha, p.n_beta, ordering).astype(np.int64)
    assert np.abs(psi_d[idx] - psi_s).max() < 1e-13
    outside = np.ones(psi_d.size, bool); outside[idx] = False
    assert np.all(psi_d[outside] == 0)
    s_d = dense.hamiltonian_apply(psi_d, p.h, p.g, 0.2, ordering)
    s_s = sector.sigma(psi_s, p.h, p.g, 0.2, p.n_alpha, p.n_beta, ordering)
    assert np.abs(s_d[idx] - s_s).max() < 1e-12
    assert np.all(s_d[outside] == 0)
    assert np.abs(dense.rdm1(psi_d, m, ordering) - sector.rdm1(psi_s, m, p.n_alpha, p.n_beta, ordering)).max() < 1e-13


# ---------------------------------------------------------------- P6 ---------
@pytest.mark.parametrize("n,ne,seed", [(12, 6, 61), (14, 7, 62)])
def test_invariants(n, ne, seed):
    p0 = random_problem(n, ne, 40, seed=seed, theta_std=0.3)
    m = p0.n_orb
    na, nb = p0.n_alpha, p0.n_beta
    res = {}
    for ordering in (0, 1):
        psi = sector.ansatz(m, na, nb, p0.ops, p0.theta, ordering)
        assert abs(np.linalg.norm(psi) - 1) < 1e-13
        assert np.abs(psi.imag).max() == 0.0
        back = sector.apply_rotations(psi, m, na, nb, p0.ops[::-1], -p0.theta[::-1], ordering)
        ref = sector.ansatz(m, na, nb, p0.ops[:0], p0.theta[:0], ordering)
        assert np.abs(back - ref).max() < 1e-13
        gam = sector.rdm1(psi, m, na, nb, ordering)
        assert abs(np.trace(gam[0]) - na) < 1e-12 and abs(np.trace(gam[1]) - nb) < 1e-12
        for s in (0, 1):
            assert np.abs(gam[s] - gam[s].conj().T).max() < 1e-14
            w = np.linalg.eigvalsh(gam[s])
            assert w.min() > -1e-12 and w.max() < 1 + 1e-12
        e, gr = sector.energy_grad(m, na, nb, p0.ops, p0.theta, p0.h, p0.g, 0.0, ordering)
        res[ordering] = (e, gr, gam)
        # linearity in the one-body potential and exact E_core shift
        v = np.random.default_rng(seed).normal(0, 0.02, (m, m)); v = v + v.T
        e_v = sector.energy(psi, p0.h + v, p0.g, 0.0, na, nb, ordering)
        assert abs((e_v - e) - np.sum(v * (gam[0] + gam[1]).real)) < 1e-12
        e_c = sector.energy(psi, p0.h, p0.g, 1.75, na, nb, ordering)
        assert abs(e_c - e - 1.75) < 1e-12
    # results do not depend on the JW qubit ordering
    assert abs(res[0][0] - res[1][0]) < 1e-12
    assert np.abs(res[0][1] - res[1][1]).max() < 1e-12
    assert np.abs(res[0][2] - res[1][2]).max() < 1e-13


# ---------------------------------------------------------------- P7 ---------
def test_variational_bound_and_exactness():
    # E(theta) >= E_FCI for any theta
    for seed in (71, 72):
        p = random_problem(10, 4, 30, seed=seed, theta_std=0.8)
        m = p.n_orb
        e_fci = brute.fci_energy(p.h, p.g, 0.0, 10, p.n_alpha, p.n_beta)
        assert abs(e_fci - sector.fci_energy(p.h, p.g, 0.0, p.n_alpha, p.n_beta)) < 1e-10
        for t in range(4):
            th = np.random.default_rng(seed * 10 + t).normal(0, 1.0, p.n_ops)
            psi = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, th)
            assert sector.energy(psi, p.h, p.g, 0.0, p.n_alpha, p.n_beta) >= e_fci - 1e-12
    # 4 spin-orbitals / 2 electrons: all-UCCSD minimum equals FCI
    p = random_problem(4, 2, None, seed=73)
    m = p.n_orb
    e_fci = brute.fci_energy(p.h, p.g, 0.0, 4, 1, 1)

    def f(th):
        return sector.energy_grad(m, 1, 1, p.ops, th, p.h, p.g, 0.0)

    best = min((scipy.optimize.minimize(f, x0, jac=True, method="BFGS", tol=1e-14)
                for x0 in (np.zeros(p.n_ops), np.full(p.n_ops, 0.5), np.full(p.n_ops, -0.7))),
               key=lambda r: r.fun)
    assert abs(best.fun - e_fci) < 1e-10


# ---------------------------------------------------------------- P8 ---------
@pytest.mark.parametrize("ordering", [0, 1])
def test_gradient_adjoint_vs_finite_difference(ordering):
    p = random_problem(10, 5, 18, seed=81, theta_std=0.4, ordering=ordering)
    m = p.n_orb
    e, gr = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, ordering)
    fd = dense.energy_fd_grad(10, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, ordering)
    assert np.abs(gr - fd).max() < 1e-6
    e2, gr2 = sector.energy_grad(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, ordering, stride=4)
    assert abs(e - e2) < 1e-13 and np.abs(gr - gr2).max() < 1e-13


def test_pool_counts():
    # UCCSD pool sizes of the five workload shapes
    assert len(uccsd_pool(4, 2, 2)) == 26
    assert len(uccsd_pool(8, 4, 4)) == 360
    assert len(uccsd_pool(12, 6, 6)) == 1818
    assert len(uccsd_pool(15, 7, 7)) == 4424
    assert len(uccsd_pool(5, 4, 3)) == 37


# ------------------------------------------------- T1 vs T3 at 16 qubits ----
@pytest.mark.parametrize("ne,seed,ordering", [(8, 57, 1), (7, 58, 0)])
def test_dense_literal_matches_sector_16q_general_integrals(ne, seed, ordering):
    # the literal 2^16 definition (every term of H applied to the qubit-basis
    # vector) against the sector tier at the size of the 16-qubit workload,
    # with (pq|rs) of full pair rank (36 random symmetric factors), so the
    # sector tier's alpha-first split of the alpha-beta term is checked on
    # integrals with no low-rank structure
    p = random_problem(16, ne, 12, seed=seed, theta_std=0.4, ordering=ordering, replace=True)
    m = p.n_orb
    rng = np.random.default_rng(seed)
    g = np.zeros((m, m, m, m))
    for _ in range(m * (m + 1) // 2):
        f = rng.normal(0, 0.05, (m, m))
        f = f + f.T
        g += np.einsum("pq,rs->pqrs", f, f)
    psi_d = dense.ansatz_state(16, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, ordering)
    idx = sector.sector_qubit_index(m, p.n_alpha, p.n_beta, ordering).astype(np.int64)
    assert np.abs(psi_d[idx] - psi_s).max() < 1e-13
    s_d = dense.hamiltonian_apply(psi_d, p.h, g, 0.3, ordering)
    s_s = sector.sigma(psi_s, p.h, g, 0.3, p.n_alpha, p.n_beta, ordering)
    assert np.abs(s_d[idx] - s_s).max() < 1e-11
    outside = np.ones(psi_d.size, bool)
    outside[idx] = False
    assert np.all(s_d[outside] == 0)


# --------------------------------------- T1 at sampled outputs, 24 qubits ----
def test_literal_hamiltonian_at_sampled_outputs_24q():
    # the 24-qubit workload's problem: the sector tier's state after its first
    # 10 operators against the literal 2^24 rotations, and its H psi at the
    # full 200-operator state against every term of H applied literally at 48
    # sampled sector outputs (the literal H psi of the whole vector is out of
    # reach at this size)
    p = config("C3")
    m = p.n_orb
    idx = sector.sector_qubit_index(m, p.n_alpha, p.n_beta, p.ordering).astype(np.int64)
    psi_d = dense.ansatz_state(24, p.n_alpha, p.n_beta, p.ops[:10], p.theta[:10], p.ordering)
    psi_s = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops[:10], p.theta[:10], p.ordering)
    assert np.abs(psi_d[idx] - psi_s).max() < 1e-13
    vec = sector.ansatz(m, p.n_alpha, p.n_beta, p.ops, p.theta, p.ordering)
    full = np.zeros(1 << 24, dtype=np.complex128)
    full[idx] = vec
    sig = sector.sigma(vec, p.h, p.g, 0.25, p.n_alpha, p.n_beta, p.ordering)
    rng = np.random.default_rng(24)
    pick = rng.choice(idx.size, 48, replace=False)
    lit = dense.hamiltonian_apply_at(full, idx[pick], p.h, p.g, 0.25, p.ordering)
    assert np.abs(lit - sig[pick]).max() < 1e-11


def test_literal_hamiltonian_at_equals_full_apply():
    # the sampled-output form of the literal H against the whole-vector form
    p = random_problem(10, 5, 12, seed=77, theta_std=0.4, ordering=1, replace=True)
    psi = dense.ansatz_state(10, p.n_alpha, p.n_beta, p.ops, p.theta, 1)
    psi = psi + 0.01 * np.random.default_rng(3).normal(size=psi.size)  # other sectors too
    xs = np.arange(psi.size)
    assert np.abs(dense.hamiltonian_apply_at(psi, xs, p.h, p.g, 0.1, 1)
                  - dense.hamiltonian_apply(psi, p.h, p.g, 0.1, 1)).max() < 1e-12
