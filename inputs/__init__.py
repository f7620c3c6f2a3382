"""Seeded synthetic inputs shared, as data, by the GPU path and the oracle.

Nothing here computes any part of the lattice Boltzmann method or the neural
operator: it builds obstacle geometries (solid mask, signed distance, wall
distance per boundary link) and seeded velocity perturbations.  Both the
product tests and the oracle read its arrays; neither side's arithmetic lives
here.
"""
from .rng import splitmix64, uniform_pm1, perturbation  # noqa: F401
from .geometry import Geometry, sphere_channel, spanwise_cylinder, random_obstacle, obstacle_sdf, from_sdf  # noqa: F401
from .features import coarse_inputs, to_bf16_bits  # noqa: F401
