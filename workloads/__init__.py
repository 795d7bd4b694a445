"""Seeded synthetic inputs for the space-time HDG + AIR solver.

This package holds only problem data: simplex meshes of the space-time
domain (vertex coordinates and cell-to-vertex lists), boundary-kind rules,
and the coefficient / exact-solution functions of each workload.  It holds
none of the method's arithmetic (no quadrature, no basis, no assembly, no
solver) and is the only code shared by the oracle and the HIP path.

Coordinates are space-time: column 0 is t, columns 1..d are space.
"""
from .meshes import (square_tri_mesh, slab_prism_tet_mesh, stacked_prism_tet_mesh, kuhn_cube_mesh,
                     map_vertices_c5, pulse_slab_mesh, boundary_kinds)
from . import problems

__all__ = ["square_tri_mesh", "slab_prism_tet_mesh", "stacked_prism_tet_mesh", "kuhn_cube_mesh",
           "map_vertices_c5", "pulse_slab_mesh", "boundary_kinds", "problems"]
