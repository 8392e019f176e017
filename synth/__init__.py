"""Seeded synthetic workloads for messenger-field mapmaking.

This package is input generation only.  It draws skies, scan patterns and
noise realisations that are shaped like the simulations of Section 2.3 of
Huffenberger & Naess (cross-linked raster scans, polarization-sensitive
detectors, white plus 1/f noise), and hands plain arrays to whichever solver
consumes them.  It contains no part of the mapmaking method itself: no noise
weighting, no filtering, no binning and no solve.

Both the CPU oracle (under ``oracle/``) and the GPU library consume the same
arrays produced here, so the two never share code beyond their inputs.
"""

from .configs import CONFIGS, WorkloadConfig, config_by_name
from .problem import Problem, make_problem

__all__ = ["CONFIGS", "WorkloadConfig", "config_by_name", "Problem", "make_problem"]
