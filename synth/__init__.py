"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only *makes inputs*: site positions, Voronoi neighbour lists with
periodic shifts and wall flags, the angle quadrature, and the per-site
temperature and density of a Bifrost-like stratified box. It computes none of
the radiative-transfer method itself (no opacities, no Planck function, no
upwind selection, no formal solution); those live separately in the oracle and
in the HIP library, which never import each other.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""

from .quadrature import gauss_legendre_quadrature, vertical_quadrature
from .atmosphere import (
    BoxSpec,
    Atmosphere,
    T0_of_z,
    rho_of_z,
    horizontal_field,
    kappa0_and_density,
    sample_sites,
    locality_order,
    make_atmosphere,
)
from .voronoi import VoronoiGrid, voronoi_neighbours, lattice_grid, check_symmetric, concat_grids

__all__ = [
    "gauss_legendre_quadrature",
    "vertical_quadrature",
    "BoxSpec",
    "Atmosphere",
    "T0_of_z",
    "rho_of_z",
    "horizontal_field",
    "kappa0_and_density",
    "sample_sites",
    "locality_order",
    "make_atmosphere",
    "VoronoiGrid",
    "voronoi_neighbours",
    "lattice_grid",
    "check_symmetric",
    "concat_grids",
    "batch_sizes",
]


def batch_sizes(n_atm: int, lo: int, hi: int, seed: int):
    """Atmosphere sizes drawn log-uniformly in [lo, hi] (rounded), seeded."""
    import numpy as _np

    rng = _np.random.Generator(_np.random.PCG64(seed))
    return [int(round(_np.exp(rng.uniform(_np.log(lo), _np.log(hi))))) for _ in range(n_atm)]
