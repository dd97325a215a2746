"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds workload descriptions and input fields only: no residual, Jacobian,
solver or functional arithmetic of the method.  Both the oracle and the HIP path are fed
the arrays produced here, so that no floating-point tie in an input recipe can make the
two sides see different problems.
"""
from .sneddon import (Workload, WORKLOADS, crack_band_phi, random_state, batched_instances, domain_study,
                      cod_study)
from .cycle import alternating_case, ALTERNATING_SEED

__all__ = ["Workload", "WORKLOADS", "crack_band_phi", "random_state", "batched_instances", "domain_study", "cod_study",
           "alternating_case", "ALTERNATING_SEED"]
