"""Seeded synthetic inputs for the cell-loop assembler and for its oracle.

This package builds *inputs only*: simplicial meshes (vertex coordinates and
cell-to-vertex Maps), cell-to-node Maps of Lagrange P1-P3 spaces, seeded P1
coefficient fields and index permutations.  It holds none of the assembly
arithmetic (no basis functions, quadrature, Jacobians or element tensors), so
the HIP library and the CPU oracle can both consume what it produces without
sharing any part of the computation they are compared on.

Meshes follow the paper's Set/Map view (Sets of vertices, cells and nodes;
constant-arity Maps between them, PyOP2 Sets and Maps sections) and its
benchmark shapes (unit square and unit cube, experiments section).
"""
from .meshes import (Mesh, unit_square, unit_cube, two_triangles, two_tets,
                     jitter_interior, node_map, permute_cells, permute_nodes,
                     permute_vertices, local_node_barycentrics, dg_coordinates,
                     flatten_cells, boundary_nodes, exterior_facets)
from .fields import field, seeds, spawn_streams

__all__ = ["Mesh", "unit_square", "unit_cube", "two_triangles", "two_tets",
           "jitter_interior", "node_map", "permute_cells", "permute_nodes",
           "permute_vertices", "local_node_barycentrics", "dg_coordinates",
           "flatten_cells", "boundary_nodes", "exterior_facets", "field", "seeds", "spawn_streams"]
