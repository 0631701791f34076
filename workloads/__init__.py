"""Seeded synthetic workloads for the periodic B-spline orbital library.

This package only draws random numbers and lays out arrays.  It holds none of
the spline method's arithmetic (no basis functions, no coefficient solves, no
evaluation), so that the FP64 oracle and the HIP library can both consume it
without sharing any of the method.

Orbitals are periodic planewave sums (the planewave expansion of the paper's
introduction, Eq. pw_orbital) with Gaussian random coefficients; their samples
on the real-space grid are taken with numpy's inverse FFT.
"""
from .synth import (
    BOHR_PER_ANGSTROM,
    System,
    make_system,
    gvectors,
    draw_coefficients,
    draw_bloch_coefficients,
    sample_grid,
    sample_grid_laplacian,
    draw_positions,
)
from .configs import CONFIGS, config, batched_systems

__all__ = [
    "BOHR_PER_ANGSTROM", "System", "make_system", "gvectors", "draw_coefficients",
    "draw_bloch_coefficients", "sample_grid", "sample_grid_laplacian", "draw_positions", "CONFIGS", "config",
    "batched_systems",
]
