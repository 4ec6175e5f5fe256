"""energy_grad_noalloc (no device allocation in the call; scratch in the
library's static per-GPU block) against energy_grad through the C ABI: two
calls in a row on different plans, the second one smaller, each to the same
bar as energy_grad against the oracle; plans beyond the block are refused."""

import ctypes

import numpy as np
import pytest

from workloads import config, random_problem
from tests.gpu_helpers import oracle_energy_grad, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsv(gpu):
    import paper_2405_11567_amd as m
    m.load()
    return m


def _noalloc(plan, theta, psi, lam):
    lib = plan._lib
    th = np.ascontiguousarray(theta, dtype=np.float64)
    grad = np.zeros(max(plan.n_ops, 1))
    e = ctypes.c_double()
    rc = lib.energy_grad_noalloc(plan._h, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(lam.data_ptr()), ctypes.byref(e),
                                 grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, e.value, grad[: plan.n_ops]


def test_noalloc_matches_energy_grad(fsv):
    # 24 qubits first, then 16 qubits (smaller): the second call meets the
    # first one's leftovers in the shared block
    for cfg in ("C3", "C2"):
        p = config(cfg)
        say("noalloc", cfg)
        plan = fsv.Plan(p)
        psi, lam = plan.new_state(), plan.new_state()
        e_ref, g_ref = plan.energy_grad(p.theta, psi, lam)
        rc, e, g = _noalloc(plan, p.theta, psi, lam)
        assert rc == 0
        assert abs(e - e_ref) < 1e-10 and np.abs(g - g_ref).max() < 1e-9
        eo, go = oracle_energy_grad(p)
        assert abs(e - eo) < 1e-10 and np.abs(g - go).max() < 1e-9
        rc2, e2, g2 = _noalloc(plan, p.theta, psi, lam)
        assert rc2 == 0 and e2 == e and np.array_equal(g2, g)


def test_noalloc_refuses_what_does_not_fit(fsv):
    # 26 qubits, 6 + 6 electrons: 2.94 M sector amplitudes need more than the block
    p = random_problem(26, 12, 10, seed=1401, theta_std=0.3, replace=True)
    plan = fsv.Plan(p)
    psi, lam = plan.new_state(), plan.new_state()
    rc, _, _ = _noalloc(plan, p.theta, psi, lam)
    assert rc == -1 and b"scratch" in plan._lib.fsv_last_error()
    dplan = fsv.Plan(config("C1"), engine="dense")
    rc, _, _ = _noalloc(dplan, config("C1").theta, dplan.new_state(), dplan.new_state())
    assert rc == -4
