"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This package builds meshes, local-to-global dof maps and coefficient nodal
values.  It holds none of the finite element method's arithmetic (no
quadrature, no basis tabulation, no geometry tensors, no element matrices,
no assembly): those live separately in the library and in the oracle.
"""
from .meshes import (  # noqa: F401
    Mesh,
    kuhn_mesh,
    jitter_interior,
    flatten_cells,
    lattice_dofmap,
    dg_dofmap,
    lattice_multi_indices,
    nodal_values,
    normal_vector,
    config_mesh,
    hex_mesh,
    DegreeBlock,
    mixed_degree_blocks,
    CONFIGS,
)
