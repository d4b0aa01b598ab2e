"""Seeded synthetic inputs for the compressible pressure solve.

This package generates permeability, porosity and well definitions with the
shapes and statistics of the paper's workloads (Sec. 4, Table "permeability
sets": log-normal fields on 64^3..256^3 grids).  It contains none of the
solver's arithmetic: it only draws random fields and describes problems.  Both
the CPU oracle tests and the GPU path consume exactly these arrays.
"""

from .fields import gaussian_field, lognormal_permeability, channel_permeability
from .configs import Problem, config1, config2, config4, config5_eval, small_problem, batch_problems

__all__ = [
    "gaussian_field",
    "lognormal_permeability",
    "channel_permeability",
    "Problem",
    "config1",
    "config2",
    "config4",
    "config5_eval",
    "small_problem",
    "batch_problems",
]
