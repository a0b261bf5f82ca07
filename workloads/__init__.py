"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package only draws meshes and rays; it contains none of the geodesic
method's arithmetic and imports neither the oracle nor the GPU library.
"""
from . import meshes, rays, configs  # noqa: F401
