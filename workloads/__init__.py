"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.  This package holds no arithmetic of the method: it only draws
integrals, excitation lists and angles from fixed seeds."""

from .synth import (  # noqa: F401
    Problem,
    synthetic_hamiltonian,
    uccsd_pool,
    config,
    batch_config,
    random_problem,
    potential_v0,
    CONFIG_NAMES,
)
