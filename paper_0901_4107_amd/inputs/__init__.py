"""Seeded input generators shared by the GPU path's tests and the oracle's.

Nothing in this package performs any step of the hydro scheme: it produces
point sets, the periodic Voronoi tessellation of those points (the given mesh
the hydro step runs on) and initial fluid states, all from fixed seeds.
"""
from .mesh import Mesh, build_mesh, morton_order  # noqa: F401
