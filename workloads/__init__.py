"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Holds no part of the numerical method: only meshes, initial data, exact
solutions and their cell averages.
"""
from .meshes import Mesh2D, split_square_mesh, unwrapped_triangles  # noqa: F401
from .problems import *  # noqa: F401,F403
