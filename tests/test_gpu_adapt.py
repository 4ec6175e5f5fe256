"""Qubit-excitation (QEB) operators and ADAPT pool screening on the GPU vs the
FP64 oracle (same tolerances as test_gpu_parity)."""

import copy

import numpy as np
import pytest

from oracle import dense, sector
from workloads import config, random_problem, uccsd_pool
from tests.gpu_helpers import dense_from_sector, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsv(gpu):
    import paper_2405_11567_amd as m
    m.load()
    return m


def _qeb(p):
    q = copy.copy(p)
    q.excitation = 1
    return q


@pytest.mark.parametrize("engine", ["sector", "dense"])
@pytest.mark.parametrize("ordering", [0, 1])
def test_qeb_ansatz_energy_grad(fsv, ordering, engine):
    # qubit excitations drawn from the whole pool (alpha-only, beta-only and
    # alpha-beta operators in both orderings: in the interleaved ordering the
    # sector signs need explicit diagonal lists)
    p = _qeb(random_problem(14, 7, 60, seed=901 + ordering, theta_std=0.5, replace=True, ordering=ordering))
    say("QEB", ordering, engine)
    plan = fsv.Plan(p, engine=engine)
    psi = plan.ansatz_apply(p.theta).cpu().numpy()
    ref, _ = dense_from_sector(sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, ordering,
                                             excitation=1), p)
    assert np.abs(psi - ref).max() < 1e-12
    e, g = plan.energy_grad(p.theta)
    e_ref, g_ref = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core,
                                      ordering, excitation=1)
    assert abs(e - e_ref) < 1e-10 and np.abs(g - g_ref).max() < 1e-9


def test_qeb_small_dense_oracle_and_fp32(fsv):
    p = _qeb(random_problem(10, 5, 25, seed=911, theta_std=0.6, replace=True, ordering=0))
    psi = fsv.Plan(p).ansatz_apply(p.theta).cpu().numpy()
    ref = dense.ansatz_state(10, p.n_alpha, p.n_beta, p.ops, p.theta, 0, excitation=1)
    assert np.abs(psi - ref).max() < 1e-12
    e, g = fsv.Plan(p, precision=1).energy_grad(p.theta)
    e_ref, g_ref = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, 0.0, 0,
                                      excitation=1)
    say("QEB FP32 |dE|", abs(e - e_ref))
    assert abs(e - e_ref) < 1e-4


@pytest.mark.parametrize("excitation", [0, 1])
@pytest.mark.parametrize("ordering", [0, 1])
def test_pool_gradients_c2(fsv, excitation, ordering):
    # the whole 360-operator pool screened at a 60-operator state
    p = config("C2", ordering=ordering)
    pool_ops = np.asarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
    p.ops, p.theta = p.ops[:60], p.theta[:60] * 4.0
    p.excitation = excitation
    say("pool C2", excitation, ordering, len(pool_ops))
    plan = fsv.Plan(p)
    pool = plan.pool(pool_ops)
    e, g = pool.gradients(p.theta)
    psi = sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, ordering, excitation)
    g_ref = sector.pool_gradients(psi, p.h, p.g, p.e_core, pool_ops, p.n_alpha, p.n_beta, ordering, excitation)
    e_ref = sector.energy(psi, p.h, p.g, p.e_core, p.n_alpha, p.n_beta, ordering)
    assert abs(e - e_ref) < 1e-10
    assert np.abs(g - g_ref).max() < 1e-9
    # replays of the captured graph are bitwise stable, with other work between
    plan.energy_grad(p.theta)
    e2, g2 = pool.gradients(p.theta)
    assert e2 == e and np.array_equal(g2, g)


def test_pool_gradients_c3_sample(fsv):
    # full-size 24-qubit state, 240 pool operators sampled from the 1818
    p = config("C3")
    full = np.asarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
    rng = np.random.default_rng(77)
    pool_ops = full[np.sort(rng.choice(len(full), 240, replace=False))]
    plan = fsv.Plan(p)
    e, g = plan.pool(pool_ops).gradients(p.theta)
    psi = sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, 0)
    g_ref = sector.pool_gradients(psi, p.h, p.g, p.e_core, pool_ops, p.n_alpha, p.n_beta, 0, 0)
    say("pool C3 max|dg|", np.abs(g - g_ref).max())
    assert np.abs(g - g_ref).max() < 1e-9
    # the full pool in one launch: the same values on the sampled operators
    e_all, g_all = plan.pool(full).gradients(p.theta)
    idx = {tuple(o): t for t, o in enumerate(full)}
    sel = np.array([idx[tuple(o)] for o in pool_ops])
    assert abs(e_all - e) < 1e-12 and np.abs(g_all[sel] - g).max() < 1e-12


def test_pool_rejects_bad_input(fsv):
    p = config("C1")
    plan = fsv.Plan(p)
    with pytest.raises(fsv.FsvError) as ei:
        plan.pool(np.array([[0, 2, 1, 3]], dtype=np.int32))  # spin flip
    assert ei.value.code == -1
    with pytest.raises(fsv.FsvError) as ei:
        plan.pool(p.ops, excitation=2)
    assert ei.value.code == -1
    dplan = fsv.Plan(p, engine="dense")
    with pytest.raises(fsv.FsvError) as ei:
        dplan.pool(p.ops)
    assert ei.value.code == -4


def test_plan_close_closes_its_pools(fsv):
    # a pool reads its plan when destroyed: closing the plan (or a garbage
    # cycle finalising it first) closes its pools before the plan
    p = config("C1")
    plan = fsv.Plan(p)
    q1, q2 = plan.pool(p.ops), plan.pool(p.ops[:5])
    e, g = q1.gradients(p.theta)
    assert np.isfinite(e) and g.shape == (p.n_ops,)
    plan.close()
    assert q1._h is None and q2._h is None and plan._h is None
    q1.close()
    plan.close()


@pytest.mark.parametrize("mode", ["phased", "persistent", "packets"])
def test_batch_qeb_instances(fsv, monkeypatch, mode):
    monkeypatch.setenv("FSV_BATCH_MODE", mode)
    probs = []
    for i, (n, ne, k) in enumerate([(10, 5, 20), (12, 6, 30), (8, 3, 15), (14, 7, 25)]):
        p = random_problem(n, ne, k, seed=920 + i, theta_std=0.4, replace=True, ordering=i % 2)
        p.excitation = (i + 1) % 2
        probs.append(p)
    b = fsv.Batch(probs)
    e, g = b.energy_grad([p.theta for p in probs])
    for i, p in enumerate(probs):
        e_ref, g_ref = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core,
                                          p.ordering, excitation=p.excitation)
        assert abs(e[i] - e_ref) < 1e-10 and np.abs(g[i] - g_ref).max() < 1e-9


def oracle_pick(g):
    # ADAPT's choice, written here independently of the product: the largest
    # screening magnitude, ties (equal after rounding to 1e-10) to the first index
    mag = np.round(np.abs(g), 10)
    best = 0
    for t in range(1, len(mag)):
        if mag[t] > mag[best]:
            best = t
    return best


def oracle_adapt(p, pool_ops, excitation, max_ops, grad_tol, inner, lr):
    pick = oracle_pick
    m, na, nb, o = p.n_orb, p.n_alpha, p.n_beta, p.ordering
    ops = np.zeros((0, 4), dtype=np.int32)
    theta = np.zeros(0)
    chosen, energies = [], []
    for _ in range(max_ops):
        psi = sector.ansatz(m, na, nb, ops, theta, o, excitation)
        g = sector.pool_gradients(psi, p.h, p.g, p.e_core, pool_ops, na, nb, o, excitation)
        k = pick(g)
        if abs(g[k]) < grad_tol:
            break
        ops = np.vstack([ops, pool_ops[k][None, :]])
        theta = np.r_[theta, 0.0]
        for _ in range(inner):
            _, gr = sector.energy_grad(m, na, nb, ops, theta, p.h, p.g, p.e_core, o, excitation=excitation)
            theta = theta - lr * gr
        e_after, _ = sector.energy_grad(m, na, nb, ops, theta, p.h, p.g, p.e_core, o, excitation=excitation)
        chosen.append(k)
        energies.append(e_after)
    return chosen, energies, theta


@pytest.mark.parametrize("excitation", [0, 1])
def test_adapt_loop_vs_oracle(fsv, excitation):
    from paper_2405_11567_amd.adapt import adapt
    p = random_problem(10, 5, None, seed=931, ordering=excitation)
    pool_ops = np.asarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
    say("ADAPT", excitation, len(pool_ops))
    res = adapt(p, pool_ops, excitation=excitation, max_ops=5, grad_tol=1e-6, inner=8, lr=0.3)
    chosen, energies, theta = oracle_adapt(p, pool_ops, excitation, 5, 1e-6, 8, 0.3)
    got = [s.chosen for s in res.steps if s.chosen >= 0]
    assert got == chosen
    assert np.abs(np.array([s.energy_after for s in res.steps if s.chosen >= 0]) - energies).max() < 1e-9
    assert np.abs(res.theta - theta).max() < 1e-8
    assert energies[-1] < energies[0]
