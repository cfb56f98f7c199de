"""Seeded synthetic inputs for the correlated-chains Monte Carlo inverter.

This package produces matrices only (CSR arrays and workload sizes).  It holds
none of the sampler's arithmetic, so both the CPU oracle and the GPU library
consume the same inputs without sharing any code path of the method.
"""

from .matrices import (  # noqa: F401
    CSR,
    random_dominant,
    pedigree,
    lattice,
    dirac,
    dirac_gammas,
    batched_sizes,
    batched_pedigrees,
    surrogate_params,
    diag_matrix,
    from_dense,
    to_dense,
    round_values,
    WORKLOADS,
)
