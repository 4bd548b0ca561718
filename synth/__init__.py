"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side tests and bench.

This package only draws numbers (permittivity fields, plane-wave directions and
polarisations, request streams).  It holds none of the method's arithmetic: no
Green's function, no compression, no solver.
"""
from .workloads import (Grid, make_grid, config, CONFIG_NAMES, random_directions,
                        random_polarisations, serving_requests)

__all__ = ["Grid", "make_grid", "config", "CONFIG_NAMES", "random_directions",
           "random_polarisations", "serving_requests"]
