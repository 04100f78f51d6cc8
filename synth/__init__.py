"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package holds no arithmetic of the method: it only draws the inputs
(eigenstrain fields, surface tractions, indenter and rough surface profiles,
request streams).  Both the HIP library's callers and the oracle receive the
arrays it returns.  Every generator takes an explicit seed and uses numpy's
PCG64 generator (``numpy.random.default_rng``).
"""
from .fields import (grid_dict, filtered_eigenstrain, filtered_traction,
                     paraboloid, rough_surface, poisson_requests)

__all__ = ["grid_dict", "filtered_eigenstrain", "filtered_traction",
           "paraboloid", "rough_surface", "poisson_requests"]
