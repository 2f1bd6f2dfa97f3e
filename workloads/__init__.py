"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Nothing in this package performs any step of the multishift solve: it only builds the
sparse operators, the shifts and the right-hand sides that both the CPU oracle and the
GPU library consume.  Every generator is a pure function of its seed.
"""
from .lattice import (
    lattice_volume,
    site_coords,
    neighbour,
    staggered_eta,
    haar_su3,
    random_su3_links,
    free_links,
    pure_gauge_links,
    staggered_csr,
)
from .generic import (laplacian7_csr, poisson5pt_csr, random_sparse_csr, gaussian_rhs,
                      logspace_shifts)
from .configs import CONFIGS, make_config, staggered_problem

__all__ = [
    "lattice_volume",
    "site_coords",
    "neighbour",
    "staggered_eta",
    "haar_su3",
    "random_su3_links",
    "free_links",
    "pure_gauge_links",
    "staggered_csr",
    "laplacian7_csr",
    "poisson5pt_csr",
    "random_sparse_csr",
    "gaussian_rhs",
    "logspace_shifts",
    "CONFIGS",
    "make_config",
    "staggered_problem",
]
