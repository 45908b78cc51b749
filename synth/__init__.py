"""Seeded synthetic inputs for both sides of every parity check.

This module only draws random numbers and lays them out as int32 buffers; it
contains none of the max-flow or assignment arithmetic.  The CPU oracle and
the HIP library both consume exactly the arrays produced here.

Every generator seeds ``numpy.random.default_rng`` with
``SeedSequence([config_id, instance_id, seed])`` (PCG64); draw order is
row-major and part of the definition of each workload.
"""
from .grids import (GridInstance, grid_uniform, grid_blobs, grid_batch,
                    grid_random_small, grid_from_pairs)
from .assign import (assign_uniform, assign_points, assign_batch,
                     assign_random_small, assign_sparse, TRAIN_BRANCH)
from .graphs import (graph_random, graph_layered, graph_bipartite, pairs_to_arcs,
                     grid_to_arcs, grid3d_arcs, grid8_arcs, mcf_random,
                     mcf_transport)

__all__ = [
    "GridInstance", "grid_uniform", "grid_blobs", "grid_batch",
    "grid_random_small", "grid_from_pairs",
    "assign_uniform", "assign_points", "assign_batch", "assign_random_small",
    "assign_sparse",
    "TRAIN_BRANCH",
    "graph_random", "graph_layered", "graph_bipartite", "pairs_to_arcs",
    "grid_to_arcs", "grid3d_arcs", "grid8_arcs", "mcf_random", "mcf_transport",
]
