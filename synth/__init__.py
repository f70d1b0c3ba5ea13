"""Seeded synthetic inputs: surface meshes, atoms and point charges.

This package holds input generation only (geometry of test surfaces and the
random draws of atoms and charges).  It contains none of the boundary-integral
method's arithmetic and is shared by the HIP path's tests/benchmarks and by the
CPU oracle alike.
"""
from .meshes import icosphere, isosurface_mesh, mesh_report, largest_component
from .charges import (ball_charges, packed_atoms_ball, packed_atoms_ellipsoid,
                      workload)

__all__ = ["icosphere", "isosurface_mesh", "mesh_report", "largest_component",
           "ball_charges", "packed_atoms_ball", "packed_atoms_ellipsoid",
           "workload"]
