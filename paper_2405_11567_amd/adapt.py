"""Host driver of the ADAPT growth loop around the GPU path.

The paper's ansätze are grown by ADAPT-VQE from a pool of excitation
operators (Computational Details: a QEB pool, qubit-excitation-based).  One
iteration:
* screen the pool at the current state psi(theta): for every pool operator T
  the energy derivative of appending exp(t T) at t = 0,
  <psi| [H, T] |psi> = 2 Re <H psi| T |psi>, all in one GPU launch;
* stop when the largest magnitude falls below `grad_tol`;
* append the operator with the largest magnitude at angle 0;
* re-optimise every angle with `inner` gradient-descent steps
  theta <- theta - lr * dE/dtheta (adjoint gradient on the GPU).

Ties in the screening magnitudes (exact spin or point-group degeneracies) are
broken by the first pool index after rounding the magnitudes to 1e-10, so the
choice does not depend on the last bits of the arithmetic.
"""

from __future__ import annotations

import copy
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class AdaptStep:
    energy: float          # E(theta) before the operator is added
    max_grad: float        # largest screening magnitude
    chosen: int            # pool index appended (-1: converged)
    energy_after: float    # E after re-optimising the angles


@dataclass
class AdaptResult:
    ops: np.ndarray
    theta: np.ndarray
    steps: List[AdaptStep] = field(default_factory=list)


def pick(grads: np.ndarray) -> int:
    return int(np.argmax(np.round(np.abs(grads), 10)))


def adapt(problem, pool_ops, excitation: int = 0, max_ops: int = 10, grad_tol: float = 1e-3,
          inner: int = 10, lr: float = 0.2, precision: int = 0, device=None) -> AdaptResult:
    """Grow an ansatz for `problem` (its own ops are ignored) from `pool_ops`
    (P x 4 {a, b, j, i}); excitation 0 fermionic, 1 qubit excitations."""
    from . import Plan

    pool_ops = np.ascontiguousarray(np.asarray(pool_ops, dtype=np.int32).reshape(-1, 4))
    prob = copy.copy(problem)
    prob.excitation = int(excitation)
    ops = np.zeros((0, 4), dtype=np.int32)
    theta = np.zeros(0)
    res = AdaptResult(ops, theta)
    for _ in range(max_ops):
        prob.ops, prob.theta = ops, theta
        plan = Plan(prob, precision=precision, device=device)
        pool = plan.pool(pool_ops, excitation)
        e, g = pool.gradients(theta)
        pool.close()
        plan.close()
        k = pick(g)
        if abs(g[k]) < grad_tol:
            res.steps.append(AdaptStep(e, float(abs(g[k])), -1, e))
            break
        ops = np.vstack([ops, pool_ops[k][None, :]])
        theta = np.r_[theta, 0.0]
        prob.ops, prob.theta = ops, theta
        plan = Plan(prob, precision=precision, device=device)
        psi, lam = plan.new_state(), plan.new_state()
        for _ in range(inner):
            _, grad = plan.energy_grad(theta, psi, lam)
            theta = theta - lr * grad
        e_after, _ = plan.energy_grad(theta, psi, lam)
        plan.close()
        res.steps.append(AdaptStep(e, float(abs(g[k])), k, e_after))
    res.ops, res.theta = ops, theta
    return res
