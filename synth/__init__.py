"""Seeded synthetic inputs shared by the library's tests/bench and by the oracle's tests.

This package holds only input generation: hexahedral meshes (vertex lattices,
connectivity, seeded vertex perturbation), per-element degrees and materials,
request streams and seeded coefficient vectors, plus the coefficient-vector
size bookkeeping both sides need to allocate buffers.  It contains none of the
discretisation's arithmetic (no basis functions, quadrature, fluxes or
projections), and it imports neither the oracle nor the library.
"""
from .meshes import (box_mesh, hanging_mesh, perturb_interior, affine_transform, centroids,
                     Mesh, trial_sizes, unknown_sizes, offsets, cube_rotations, reorient)
from .configs import (cavity_small, cavity_two_material, graded_nonaffine,
                      serving_stream, large_cavity, local_time_cavity, random_vector, Source,
                      ModeSet)

__all__ = [
    "box_mesh", "hanging_mesh", "perturb_interior", "affine_transform", "centroids", "Mesh",
    "cube_rotations", "reorient",
    "trial_sizes", "unknown_sizes", "offsets", "cavity_small",
    "cavity_two_material", "graded_nonaffine", "serving_stream",
    "large_cavity", "local_time_cavity", "random_vector", "Source", "ModeSet",
]
