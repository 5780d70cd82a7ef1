"""Seeded synthetic inputs shared by the oracle's tests and the GPU path's callers.

This package holds problem definitions only: physical constants, the five
workload configurations and the synthetic potential-energy surfaces the
preparatory stage would evaluate.  It contains none of the propagation
method's arithmetic (no grids, quadratures, kinetic operators, recursion or
analysis); each side builds its own from these plain parameters.
"""
from .constants import EH_EV, AMU_ME, ANG_BOHR, ev, amu  # noqa: F401
from .configs import CONFIGS, config, small_variant  # noqa: F401
from .pes import diabatic_matrix, asymptotic_potential  # noqa: F401
