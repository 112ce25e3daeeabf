"""Seeded synthetic mixTS-PIMD systems (positions, momenta, topology, force field).

This package only *draws* inputs: coordinates, momenta and parameter tables.
It holds none of the method's arithmetic (no forces, energies, normal modes or
propagation), so that the CPU oracle and the GPU library can both consume its
output without sharing any computational code.
"""
from .systems import (  # noqa: F401
    System,
    solvated_electron,
    water_box,
    tiny_random,
    config_c1,
    config_c2,
    config_c3,
    config_c4_states,
    config_c5,
    build_workers,
    water_bead_total,
)
