"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds input data (lattice frame series, their analytic
ground-truth displacements) and holds the workload constants.  It contains no
part of the registration method's arithmetic: neither the oracle nor the HIP
library imports anything from the other, both import from here.
"""
from .configs import CONFIGS, RIGID_TAU, SolverParams, SeriesSpec, get_config
from .lattice import Series, clean_frame, make_series, ground_truth, lattice_image, rigid_pair, rigid_series, RigidSeries

__all__ = ["CONFIGS", "SolverParams", "SeriesSpec", "get_config", "Series",
           "make_series", "ground_truth", "lattice_image", "clean_frame", "rigid_pair",
           "rigid_series", "RigidSeries", "RIGID_TAU"]
