"""Host driver of the Strategy-2 self-consistent loop around the GPU path.

Strategy 2 (self-consistent basis-set correction) alternates:
* solve the ansatz for the effective Hamiltonian H + V[n];
* compute the one-particle density matrix of the ansatz state (Strategy 2,
  density-matrix equation);
* classically rebuild the one-body potential from it.

The paper stops when two successive energy eigenvalues differ by less than
0.1 mHa, which takes about 2 iterations. It then reports
E2 = E + Ebar[n] - integral(v n) + dE_HF.

The density functional that produces the potential is not in the paper (it is
PBE-based and needs a real-space grid).  A stand-in with the same interface
replaces it:
    Ebar[gamma] = tr(V0 gamma) + kappa/2 ||gamma - gamma_ref||_F^2
    v           = dEbar/dgamma = V0 + kappa (gamma - gamma_ref)
where gamma is the spin-summed real density matrix and gamma_ref that of the
reference determinant.  kappa = 0 makes v a fixed potential.

Each outer iteration does the following:
* set v;
* take `inner` gradient-descent steps theta <- theta - lr * grad E on the GPU;
* compute the energy and the 1-RDM;
* record E2 = E + Ebar - tr(v gamma).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


def reference_density(n_orb: int, n_alpha: int, n_beta: int) -> np.ndarray:
    d = np.zeros(n_orb)
    d[:n_alpha] += 1.0
    d[:n_beta] += 1.0
    return np.diag(d)


@dataclass
class SCRecord:
    iteration: int
    energy: float
    e2: float
    delta: float
    gamma: np.ndarray
    theta: np.ndarray
    v: np.ndarray


@dataclass
class SCResult:
    records: List[SCRecord] = field(default_factory=list)
    first_converged: int | None = None  # first iteration with |dE| < threshold


def self_consistent_loop(plan, theta0, v0, n_alpha: int, n_beta: int, kappa: float = 0.0,
                         outer: int = 10, inner: int = 5, lr: float = 0.1,
                         threshold: float = 1e-4, psi=None, lam=None) -> SCResult:
    """Run the loop on a Plan (energy_grad, ansatz_apply, energy, rdm1 and
    set_onebody_potential all run on the GPU).  Returns per-iteration records."""
    m = plan.n_orb
    g_ref = reference_density(m, n_alpha, n_beta)
    theta = np.array(theta0, dtype=np.float64)
    psi = plan.new_state() if psi is None else psi
    lam = plan.new_state() if lam is None else lam
    plan.set_onebody_potential(None)
    plan.ansatz_apply(theta, psi)
    gam = plan.rdm1(psi)
    res = SCResult()
    e_prev = None
    for it in range(outer):
        gsum = (gam[0] + gam[1]).real
        v = v0 + kappa * (gsum - g_ref)
        plan.set_onebody_potential(v)
        for _ in range(inner):
            _, g = plan.energy_grad(theta, psi, lam)
            theta = theta - lr * g
        plan.ansatz_apply(theta, psi)
        e = plan.energy(psi)
        gam = plan.rdm1(psi)
        gsum = (gam[0] + gam[1]).real
        ebar = float(np.sum(v0 * gsum) + 0.5 * kappa * np.sum((gsum - g_ref) ** 2))
        e2 = e + ebar - float(np.sum(v * gsum))
        delta = float("nan") if e_prev is None else e - e_prev
        if res.first_converged is None and e_prev is not None and abs(delta) < threshold:
            res.first_converged = it
        res.records.append(SCRecord(it, e, e2, delta, gam, theta.copy(), v))
        e_prev = e
    plan.set_onebody_potential(None)
    return res
