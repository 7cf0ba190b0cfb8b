"""FP64 CPU oracle for the double-MRT lattice Boltzmann phase-change step.

Test infrastructure only: the tests, the package smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never does.
"""
from .oracle import (OracleSim, build, make_params, lattice, feq, meq, force_moments, geq,
                     neq, collide_f, closure, enthalpy, ke, derive, default_params)

__all__ = ["OracleSim", "build", "make_params", "lattice", "feq", "meq", "force_moments",
           "geq", "neq", "collide_f", "closure", "enthalpy", "ke", "derive",
           "default_params"]
