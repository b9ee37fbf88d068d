"""Seeded synthetic inputs for the spherical-shell conduction / viscosity workloads.

This package only *generates inputs*: grid face coordinates, temperature,
magnetic unit vectors and velocity components.  It holds none of the
method's arithmetic (no diffusivity, geometry factors, fluxes, time
stepping or solves), so that both the CPU oracle and the GPU library can
consume the same arrays without sharing any computation.  cnn_init draws the
learned-guess network's initial weights.
"""
from .shell import (  # noqa: F401
    WORKLOADS,
    Workload,
    shell_faces,
    box_faces,
    smooth_noise,
    temperature,
    dipole_bhat,
    velocity,
    make_workload,
    random_unit_vectors,
    edge_potential,
)
from .cnn_init import he_normal, flatten, unflatten, layer_dims  # noqa: F401,E402
