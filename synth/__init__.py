"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This package holds random-number generation, random-field filtering and the
workload recipes (grid sizes, constitutive parameters, boundary data, initial
heads, solver controls).  It holds none of the method's arithmetic: no
constitutive law, no residual, no Jacobian, no solver.  Both the oracle and the
HIP path receive the arrays produced here as plain inputs.
"""
from .fields import splitmix64, uniform01, std_normal, gaussian_field, lognormal_ks
from .configs import (Problem, Options, Recipe, recipe, RECIPES, serving_stream, cube_problem, MEAN_NAMES,
                      ARITH, UPSTREAM, HARMONIC, GEOMETRIC, INTEGRAL, NOFLUX, DIRICHLET, FP64, MIXED,
                      KS0, P_INIT, P_TOP, L_CUBE)
