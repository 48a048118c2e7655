"""Seeded synthetic inputs shared by the oracle and the device path (data only)."""
from .mesh import SurfaceMesh, cube_surface, icosphere, jerusalem_cross, square_plate, rwg_table, vertex_triangles
from .configs import (ETA0, K0, Workload, Request, make_workload, serving_trace, rng, standard_mom_workload,
                      element_mesh,
                      synthetic_macromodels, synthetic_d_matrix, d_pattern)
