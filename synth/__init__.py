"""Seeded synthetic particle systems, the inputs that both the HIP path and the
oracle consume.  This package draws inputs only: it holds none of the method's
arithmetic (no skins, lists, forces or integration)."""
from .systems import (CONFIGS, ParticleSystem, config_systems, free_flight_system,
                      hopper_system, incline_system, lattice_system, physics_constants,
                      silo_system)

__all__ = ["CONFIGS", "ParticleSystem", "config_systems", "free_flight_system",
           "hopper_system", "incline_system", "lattice_system", "physics_constants",
           "silo_system"]
