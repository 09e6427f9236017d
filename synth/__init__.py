"""Seeded synthetic inputs (cells and Gaussian basis sets) shared by the
oracle tests, the GPU tests and the benchmark.

This package holds input generation only: geometry, exponent and coefficient
draws and the normalisation of contracted shells.  None of the integral
method's arithmetic lives here.
"""
from .configs import (  # noqa: F401
    Basis,
    Cell,
    Problem,
    config1,
    config2,
    config3,
    config4_cells,
    config5,
    tiny_problem,
    nacl_problem,
    NACL_CHARGES,
    supercell,
    cart_count,
)
