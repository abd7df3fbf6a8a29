"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds workload numbers (``configs``) and random inputs (``screens``);
it computes none of the sensor model.
"""
from . import configs, screens  # noqa: F401
