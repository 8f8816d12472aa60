"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package generates *inputs only*: triangle meshes (vertex coordinates and
vertex-index triples, cell order) and the parameter vectors of the initial-value
problems.  It contains none of the DG method's arithmetic (no basis functions,
quadrature, fluxes, OE or limiter); both the oracle and the HIP library build
their own edge tables, geometry and projections from what is generated here.
"""

from .rng import Stream
from .mesh import (
    Mesh,
    periodic_jittered_grid,
    poisson_delaunay,
    hilbert_order,
)
from .problems import (
    PROBLEM_VORTEX,
    PROBLEM_QUADRANT,
    PROBLEM_BLAST,
    PROBLEM_TWO_STATE,
    vortex_params,
    quadrant_riemann_params,
    blast_params,
    two_state_params,
    vortex_exact_primitive,
)
from . import workloads

__all__ = [
    "Stream",
    "Mesh",
    "periodic_jittered_grid",
    "poisson_delaunay",
    "hilbert_order",
    "PROBLEM_VORTEX",
    "PROBLEM_QUADRANT",
    "PROBLEM_BLAST",
    "PROBLEM_TWO_STATE",
    "vortex_params",
    "quadrant_riemann_params",
    "blast_params",
    "two_state_params",
    "vortex_exact_primitive",
    "workloads",
]
