"""Strategy-2 loop on the GPU vs the same loop run on the oracle: energies,
density matrices and parameters per outer iteration."""

import numpy as np
import pytest

from oracle import sector
from workloads import config, potential_v0
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def oracle_loop(p, v0, kappa, outer, inner, lr):
    m, na, nb = p.n_orb, p.n_alpha, p.n_beta
    g_ref = np.diag(np.r_[np.ones(na), np.zeros(m - na)] + np.r_[np.ones(nb), np.zeros(m - nb)])
    theta = p.theta.copy()
    psi = sector.ansatz(m, na, nb, p.ops, theta, p.ordering)
    gam = sector.rdm1(psi, m, na, nb, p.ordering)
    out = []
    for _ in range(outer):
        gsum = (gam[0] + gam[1]).real
        v = v0 + kappa * (gsum - g_ref)
        for _ in range(inner):
            _, g = sector.energy_grad(m, na, nb, p.ops, theta, p.h + v, p.g, p.e_core, p.ordering)
            theta = theta - lr * g
        psi = sector.ansatz(m, na, nb, p.ops, theta, p.ordering)
        e = sector.energy(psi, p.h + v, p.g, p.e_core, na, nb, p.ordering)
        gam = sector.rdm1(psi, m, na, nb, p.ordering)
        out.append((e, gam, theta.copy()))
    return out


@pytest.mark.parametrize("cfg,kappa,outer,inner", [("C2", 0.0, 4, 5), ("C2", 0.05, 4, 5), ("C3", 0.0, 2, 2)])
def test_scloop_matches_oracle(gpu, cfg, kappa, outer, inner):
    import paper_2405_11567_amd as fsv
    from paper_2405_11567_amd.scloop import self_consistent_loop
    p = config(cfg)
    v0 = potential_v0(p.n_orb, seed=33)
    say("scloop", cfg, kappa, outer)
    plan = fsv.Plan(p)
    res = self_consistent_loop(plan, p.theta, v0, p.n_alpha, p.n_beta, kappa=kappa, outer=outer,
                               inner=inner)
    ref = oracle_loop(p, v0, kappa, outer, inner, 0.1)
    for rec, (e, gam, th) in zip(res.records, ref):
        assert abs(rec.energy - e) < 1e-10
        assert np.abs(rec.gamma - gam).max() < 1e-9
        assert np.abs(rec.theta - th).max() < 1e-9
    es = [r.energy for r in res.records]
    say("  energies", ["%.8f" % x for x in es], "first |dE|<1e-4 at", res.first_converged)
    if kappa == 0.0:
        assert es[-1] < es[0]  # gradient descent on a fixed Hamiltonian lowers the energy
