"""Seeded synthetic inputs (meshes, densities, leaf boxes) for the Q2X tests,
benchmark and smoke check.  Holds no part of the Q2X arithmetic; shared by the
GPU path's tests and the oracle's tests alike."""
from . import configs, meshes, octree  # noqa: F401
