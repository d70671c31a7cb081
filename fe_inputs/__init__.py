"""Seeded synthetic inputs shared by the oracle-side tests and the device path.

This package only generates connectivity, element matrices, size mixes and
arrival times.  It contains none of the assembly arithmetic.
"""
from . import configs, matrices, meshes  # noqa: F401
