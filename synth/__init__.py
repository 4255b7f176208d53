"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws random numbers and turns them into integer capacity
arrays.  It holds none of the max-flow arithmetic: neither the solver nor the
oracle lives here, and it imports neither of them.
"""
from .grids import (  # noqa: F401
    OFFSETS_2D4, OFFSETS_2D8, OFFSETS_3D6, offsets_for, GridInstance,
    blob_grid, config, config3_instances, random_grid, paper_e1_grid,
    random_digraph,
)
from .graphs import (  # noqa: F401
    GraphInstance, random_graph, grid26_graph, block_regions, index_regions, random_regions,
)
