"""Seeded synthetic inputs for the adaptive-multilevel BDDC solver.

This package only draws inputs (coefficient fields, substructure partitions,
level agglomerations, right-hand sides).  It holds none of the method's
arithmetic, so both the CPU oracle and the GPU library may use it.
"""

from .configs import (  # noqa: F401
    Problem,
    square_partition,
    square_agglomeration,
    add_channels,
    square_problem,
    voronoi_partition,
    voronoi_agglomeration,
    voronoi_problem,
    jag_edge,
    paper_elasticity_problem,
    config,
    request_stream, serving_stream,
    CONFIG_NAMES,
)
