"""Seeded synthetic inputs shared by the solver's tests/bench and the oracle.

Only input construction lives here (random streams, stencil matrices and
right-hand sides); none of the solver's arithmetic does.
"""
from .prng import splitmix64, splitmix64_scalar, uniform01, uniform_pm1, uniform_int, he_uniform_params  # noqa: F401
from .stencils import (CSR, laplace2d, laplace3d, convdiff2d,  # noqa: F401
                       nnz_closed_form_2d, nnz_closed_form_3d, laplacian_eigs_closed_form)
from .configs import *  # noqa: F401,F403
