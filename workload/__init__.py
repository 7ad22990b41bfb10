"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package holds only input generation (random parameters, the log-normal
coefficient field, the right-hand side, observation sites and noise).  It holds
none of the solver's arithmetic, and neither the oracle nor the GPU library is
imported from here.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    edge_sites,
    off_tree_rects,
    Workload,
    kl_modes,
    kappa_from_q,
    make_workload,
    coefficient_field,
    rhs_nodal,
    paper_kappa,
)
