"""Seeded synthetic inputs shared by the oracle and the device path (data only)."""
from .mesh import SurfaceMesh, cube_surface, square_plate, rwg_table, vertex_triangles
from .configs import (ETA0, K0, Workload, Request, make_workload, serving_trace, rng,
                      synthetic_macromodels, synthetic_d_matrix, d_pattern)
