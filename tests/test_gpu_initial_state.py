"""Multi-determinant initial states and one-body properties on the GPU vs the
FP64 oracle (same tolerances as test_gpu_parity)."""

import numpy as np
import pytest

from oracle import sector
from workloads import config, random_problem, uccsd_pool
from tests.gpu_helpers import dense_from_sector, random_dets, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsv(gpu):
    import paper_2405_11567_amd as m
    m.load()
    return m


@pytest.mark.parametrize("engine", ["sector", "dense"])
@pytest.mark.parametrize("ordering", [0, 1])
def test_multideterminant_start_c2(fsv, ordering, engine):
    p = config("C2", ordering=ordering)
    dets, coef = random_dets(p, 50, 1000 + ordering)
    psi0 = sector.determinants_vector(p.n_orb, p.n_alpha, p.n_beta, dets, coef, ordering)
    say("multi-det C2", ordering, engine)
    plan = fsv.Plan(p, engine=engine)
    plan.set_initial_state(dets, coef)
    psi = plan.ansatz_apply(p.theta).cpu().numpy()
    ref, _ = dense_from_sector(sector.apply_rotations(psi0, p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta,
                                                      ordering), p)
    assert np.abs(psi - ref).max() < 1e-12
    e, g = plan.energy_grad(p.theta)
    e_ref, g_ref = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core,
                                      ordering, psi0=psi0)
    assert abs(e - e_ref) < 1e-10 and np.abs(g - g_ref).max() < 1e-9
    e_fd, g_fd = plan.energy_grad_fd(p.theta, 1e-5)
    assert abs(e_fd - e_ref) < 1e-10 and np.abs(g_fd - g).max() < 1e-6
    # back to the reference determinant
    plan.set_initial_state()
    e0, _ = plan.energy_grad(p.theta)
    e0_ref, _ = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, ordering)
    assert abs(e0 - e0_ref) < 1e-10


def test_multideterminant_start_c3_and_pool(fsv):
    p = config("C3")
    dets, coef = random_dets(p, 300, 1010)
    psi0 = sector.determinants_vector(p.n_orb, p.n_alpha, p.n_beta, dets, coef, 0)
    plan = fsv.Plan(p)
    plan.set_initial_state(dets, coef)
    e, g = plan.energy_grad(p.theta)
    e_ref, g_ref = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, 0,
                                      psi0=psi0)
    say("multi-det C3 |dE|", abs(e - e_ref), "max|dg|", np.abs(g - g_ref).max())
    assert abs(e - e_ref) < 1e-10 and np.abs(g - g_ref).max() < 1e-9
    full = np.asarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
    pool_ops = full[::9]
    e2, gp = plan.pool(pool_ops).gradients(p.theta)
    psi = sector.apply_rotations(psi0, p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, 0)
    gp_ref = sector.pool_gradients(psi, p.h, p.g, p.e_core, pool_ops, p.n_alpha, p.n_beta, 0, 0)
    assert abs(e2 - e_ref) < 1e-10 and np.abs(gp - gp_ref).max() < 1e-9


@pytest.mark.parametrize("ordering", [0, 1])
def test_onebody_expectation(fsv, ordering):
    p = config("C2", ordering=ordering)
    plan = fsv.Plan(p)
    psi = plan.ansatz_apply(p.theta)
    rng = np.random.default_rng(5)
    d = rng.normal(size=(p.n_orb, p.n_orb))
    val = plan.onebody_expectation(psi, d)
    gam = sector.rdm1(sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, ordering), p.n_orb,
                      p.n_alpha, p.n_beta, ordering)
    ref = np.sum(d * (gam[0] + gam[1]))
    assert abs(val - ref) < 1e-11
    ds = d + d.T  # symmetric (a dipole component): real value
    assert abs(plan.onebody_expectation(psi, ds).imag) < 1e-14


def test_initial_state_rejects_bad_input(fsv):
    p = random_problem(10, 5, 6, seed=3)
    plan = fsv.Plan(p)
    idx = sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, 0).astype(np.uint64)
    with pytest.raises(fsv.FsvError) as ei:
        plan.set_initial_state([int(idx[0]) | (1 << 9) | (1 << 7)], [1.0])  # wrong electron count
    assert ei.value.code == -1
    with pytest.raises(fsv.FsvError) as ei:
        plan.set_initial_state([idx[1], idx[1]], [0.6, 0.8])
    assert ei.value.code == -1
    with pytest.raises(fsv.FsvError) as ei:
        plan.set_initial_state([idx[1]], [np.nan])
    assert ei.value.code == -5
    # a failed call leaves the previous start in place
    e, _ = plan.energy_grad(p.theta)
    e_ref, _ = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, 0)
    assert abs(e - e_ref) < 1e-10
