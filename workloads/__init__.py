"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package builds meshes and random initial states and nothing else: it
holds none of the partition method's arithmetic, so it can feed both sides of
a parity comparison without coupling them.
"""
from .meshes import (icosahedron, icosphere, torus, ellipsoid, surface_d,  # noqa: F401
                     surface_mesh, MESH_KINDS, project_sphere, project_ellipsoid,
                     project_surface_d, surface_d_phi)
from .states import (uniform_u0, one_hot_u0, batch_u0, poisson_trace,  # noqa: F401
                     eps_study_levels)
