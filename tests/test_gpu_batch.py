"""Batched path (phased launches and the persistent work-queue kernel) vs the
FP64 oracle, instance by instance."""

import time

import numpy as np
import pytest

from workloads import batch_config, random_problem
from oracle import sector
from tests.gpu_helpers import oracle_energy_grad, random_dets, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsv(gpu):
    import paper_2405_11567_amd as m
    m.load()
    return m


@pytest.mark.parametrize("same_spin", ["dense", "sparse"])
@pytest.mark.parametrize("sigma", ["lds", "direct", "global"])
@pytest.mark.parametrize("mode", ["phased", "persistent", "packets"])
def test_batch_mixed_small(fsv, mode, sigma, same_spin, monkeypatch):
    # H C with rows staged in LDS (the alpha-beta term through the factors of
    # (pq|rs) where that is exact and cheaper, or directly), and from global
    # memory only (the path taken by rows too long for LDS); same-spin parts on
    # the matrix cores (instances of at least 16 x 16 strings: 20 x 20, 35 x 35,
    # 56 x 70 here, so partial tiles and inner dimensions) or as sparse rows
    monkeypatch.setenv("FSV_BATCH_MODE", mode)
    if sigma != "lds":
        monkeypatch.setenv("FSV_BATCH_SIGMA", sigma)
    if same_spin == "sparse":
        monkeypatch.setenv("FSV_BATCH_SAME_SPIN", "sparse")
    probs = []
    shapes = [(4, 2, 3), (6, 3, 10), (8, 4, 26), (8, 1, 5), (10, 7, 20), (12, 6, 40), (12, 4, 30),
              (10, 5, 0), (14, 7, 25), (6, 6, 0), (16, 9, 30)]
    for i, (n, ne, k) in enumerate(shapes):
        p = random_problem(n, ne, k if k else None, seed=700 + i, theta_std=0.3, replace=True,
                           ordering=i % 2)
        if k == 0:
            p.ops = np.zeros((0, 4), dtype=np.int32)
            p.theta = np.zeros(0)
        p.e_core = 0.1 * i
        probs.append(p)
    say("batch mixed", len(probs), mode, sigma, same_spin)
    b = fsv.Batch(probs)
    e, g = b.energy_grad([p.theta for p in probs])
    for i, p in enumerate(probs):
        e_ref, g_ref = oracle_energy_grad(p)
        assert abs(e[i] - e_ref) < 1e-10, (i, e[i], e_ref)
        if p.n_ops:
            assert np.abs(g[i] - g_ref).max() < 1e-9, i


@pytest.mark.parametrize("mode", ["phased", "persistent", "packets"])
def test_batch_c4_full(fsv, mode, monkeypatch):
    monkeypatch.setenv("FSV_BATCH_MODE", mode)
    probs = batch_config()
    say("batch C4: 256 instances", mode)
    b = fsv.Batch(probs)
    thetas = [p.theta for p in probs]
    e, g = b.energy_grad(thetas)
    t0 = time.time()
    worst_e = worst_g = 0.0
    for i, p in enumerate(probs):
        e_ref, g_ref = oracle_energy_grad(p)
        worst_e = max(worst_e, abs(e[i] - e_ref))
        worst_g = max(worst_g, float(np.abs(g[i] - g_ref).max()))
    say(f"  oracle {time.time() - t0:.1f} s, max|dE| {worst_e:.2e}, max|dg| {worst_g:.2e}")
    assert worst_e < 1e-10 and worst_g < 1e-9
    e2, g2 = b.energy_grad(thetas)
    assert np.array_equal(e, e2) and all(np.array_equal(a, c) for a, c in zip(g, g2))
    ef, gf = b.energy_grad(np.concatenate(thetas))  # flat angles in, flat gradients out
    assert np.array_equal(ef, e) and np.array_equal(gf, np.concatenate(g))
    rep = b.autotune()
    say(rep)
    e3, g3 = b.energy_grad(thetas)
    assert np.abs(e3 - e).max() < 1e-12


def test_batch_rejects_bad_input(fsv):
    p = random_problem(8, 4, 5, seed=1)
    with pytest.raises(fsv.FsvError):
        fsv.Batch([])
    b = fsv.Batch([p])
    with pytest.raises(fsv.FsvError) as ei:
        b.energy_grad([np.full(5, np.inf)])
    assert ei.value.code == -5


def _oracle_from(p, dets, coef):
    psi0 = sector.determinants_vector(p.n_orb, p.n_alpha, p.n_beta, dets, coef, p.ordering)
    return sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, p.ordering,
                              psi0=psi0, excitation=getattr(p, "excitation", 0))


@pytest.mark.parametrize("mode", ["phased", "persistent", "packets"])
def test_batch_multideterminant_starts(fsv, mode, monkeypatch):
    # some instances start from multi-determinant states (both orderings,
    # fermionic and qubit excitations), the rest from their reference; then a
    # list is replaced by a longer one, another cleared, and bad input refused
    monkeypatch.setenv("FSV_BATCH_MODE", mode)
    shapes = [(8, 4, 12), (10, 5, 20), (12, 6, 30), (12, 5, 25), (14, 7, 18), (16, 8, 22)]
    probs = []
    for i, (n, ne, k) in enumerate(shapes):
        p = random_problem(n, ne, k, seed=1500 + i, theta_std=0.3, replace=True, ordering=i % 2)
        p.excitation = 1 if i == 3 else 0
        probs.append(p)
    say("batch multi-det", mode)
    b = fsv.Batch(probs)
    starts = {1: random_dets(probs[1], 20, 11), 2: random_dets(probs[2], 40, 12), 3: random_dets(probs[3], 7, 13),
              5: random_dets(probs[5], 60, 15)}
    for i, (d, c) in starts.items():
        b.set_initial_state(i, d, c)
    thetas = [p.theta for p in probs]

    def check():
        e, g = b.energy_grad(thetas)
        for i, p in enumerate(probs):
            if i in starts:
                e_ref, g_ref = _oracle_from(p, *starts[i])
            else:
                e_ref, g_ref = oracle_energy_grad(p)
            assert abs(e[i] - e_ref) < 1e-10, (i, e[i], e_ref)
            assert np.abs(g[i] - g_ref).max() < 1e-9, i

    check()
    starts[2] = random_dets(probs[2], 90, 22)
    b.set_initial_state(2, *starts[2])
    del starts[5]
    b.set_initial_state(5)
    check()
    with pytest.raises(fsv.FsvError) as ei:
        b.set_initial_state(len(probs), *random_dets(probs[0], 3, 1))
    assert ei.value.code == -1
    bad = np.array([np.uint64(1)], dtype=np.uint64)  # one electron: outside every sector here
    with pytest.raises(fsv.FsvError) as ei:
        b.set_initial_state(0, bad, [1.0])
    assert ei.value.code == -1
    d, c = random_dets(probs[0], 4, 3)
    with pytest.raises(fsv.FsvError) as ei:
        b.set_initial_state(0, np.r_[d, d[:1]], np.r_[c, c[:1]])
    assert ei.value.code == -1
    check()  # refused calls leave the lists as they were
