"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Meshes (geometry and region labels), material tables and source currents.
This package holds none of the finite-element method's arithmetic.
"""
from .meshes import Mesh, box, cube, cylinder, tube, tube_materials, ring_triangulation, extrude, perturbed_tube  # noqa: F401
from .sources import grad_cross, cube_current, coil_current, probe_currents, solenoid_current  # noqa: F401
