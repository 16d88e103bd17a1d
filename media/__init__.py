"""Seeded synthetic fractured media: the inputs both the oracle and the GPU path consume.

This package holds only input recipes (grids, permeability fields, fracture geometry,
boundary data, initial states).  It contains none of the finite-volume or time-stepping
arithmetic of the method: transmissibilities, storage terms, transfer assembly and every
solve are computed separately by the oracle and by the HIP library from these arrays.
"""
from .problem import OmegaContinuum, Problem, BC_NOFLOW, BC_DIRICHLET
from .configs import (config_problem, CONFIG_NAMES, small_problem, rect_problem,
                      c4_problems, c5_trace, lognormal_field, paper_problem,
                      box_problem)

__all__ = ["OmegaContinuum", "Problem", "BC_NOFLOW", "BC_DIRICHLET", "config_problem",
           "CONFIG_NAMES", "small_problem", "rect_problem", "c4_problems", "c5_trace", "lognormal_field",
           "paper_problem", "box_problem"]
