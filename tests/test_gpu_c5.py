"""30-qubit workload (C5) at full size vs stored oracle values.

The oracle needs minutes of CPU time at this size, so its energy, gradient,
1-RDM and a sample of 64 state amplitudes are stored in
tests/golden/c5_oracle.json by tests/golden/make_golden.py (which calls only
the oracle and the input generators)."""

import json
import os

import numpy as np
import pytest

from workloads import config
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_c5_sector_engine(gpu, golden):
    import paper_2405_11567_amd as fsv
    p = config("C5")
    say("C5 sector engine: energy + adjoint gradient, 1-RDM, sampled amplitudes")
    plan = fsv.Plan(p)
    psi, lam = plan.new_state(), plan.new_state()
    e, g = plan.energy_grad(p.theta, psi, lam)
    say("  E", e, golden["energy"], "max|dg|", np.abs(g - np.array(golden["grad"])).max())
    assert abs(e - golden["energy"]) < 1e-10
    assert np.abs(g - np.array(golden["grad"])).max() < 1e-9
    plan.ansatz_apply(p.theta, psi)
    idx = np.array(golden["sample_index"], dtype=np.int64)
    amp = psi[idx].cpu().numpy()
    assert np.abs(amp.real - np.array(golden["sample_amplitude"])).max() < 1e-12
    assert np.abs(amp.imag).max() == 0.0
    gam = plan.rdm1(psi)
    assert np.abs(gam[0].real - np.array(golden["gamma_alpha_real"])).max() < 1e-9
    assert np.abs(gam[1].real - np.array(golden["gamma_beta_real"])).max() < 1e-9
    assert abs(plan.energy(psi) - golden["energy"]) < 1e-10


def test_c5_dense_engine_energy(gpu, golden):
    import paper_2405_11567_amd as fsv
    p = config("C5")
    say("C5 dense engine: energy + adjoint gradient")
    plan = fsv.Plan(p, engine="dense")
    e, g = plan.energy_grad(p.theta)
    assert abs(e - golden["energy"]) < 1e-10
    assert np.abs(g - np.array(golden["grad"])).max() < 1e-9
