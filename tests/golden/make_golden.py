"""Write oracle reference values for the 30-qubit workload (C5) to
tests/golden/c5_oracle.json.  Calls only the oracle and the input generators;
the GPU tests compare against the stored numbers because the oracle needs
minutes of CPU time at this size.

Usage: python tests/golden/make_golden.py
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sector  # noqa: E402
from workloads import config  # noqa: E402


def main():
    p = config("C5")
    t0 = time.time()
    e, g = sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core,
                              p.ordering)
    t1 = time.time()
    psi = sector.ansatz(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.ordering)
    gam = sector.rdm1(psi, p.n_orb, p.n_alpha, p.n_beta, p.ordering)
    rng = np.random.default_rng(55)
    idx = np.sort(rng.choice(psi.size, 64, replace=False))
    xq = sector.sector_qubit_index(p.n_orb, p.n_alpha, p.n_beta, p.ordering)
    out = {
        "config": "C5: 30 qubits, 14 electrons, 500 operators (seed 5), ordering 0, e_core 0",
        "source": "oracle/sector.c energy_grad (stored-state adjoint) and rdm1, FP64",
        "energy": e,
        "grad": g.tolist(),
        "gamma_alpha_real": gam[0].real.tolist(),
        "gamma_beta_real": gam[1].real.tolist(),
        "sample_index": [int(xq[i]) for i in idx],
        "sample_amplitude": [float(psi[i].real) for i in idx],
        "oracle_seconds": t1 - t0,
        "threads": sector.num_threads(),
    }
    path = os.path.join(ROOT, "tests", "golden", "c5_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: E = {e:.15f}, {t1 - t0:.0f} s on {out['threads']} threads")


if __name__ == "__main__":
    main()
