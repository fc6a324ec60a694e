"""Seeded synthetic initial conditions.

This package is the only code that both the oracle and the HIP path use: it
draws particle masses, positions and velocities and holds none of the
integrator's arithmetic.
"""
from .orbits import elements_to_cartesian, solve_kepler, to_barycentric  # noqa: F401
from .configs import (  # noqa: F401
    kepler_two_body, ring64, disc16k, plummer_cluster, batch_systems, large_disc, disc100, CONFIGS,
)
