"""MI355X-native CPR (Correction Procedure via Reconstruction) hot path for
the 2D Euler equations: a C-ABI HIP library (libcpr.so, include/cpr.h) and
its thin Python binding.

    from paper_1709_01619_amd import Solver, Rollout
"""

from .solver import Rollout, Solver  # noqa: F401
from . import _lib  # noqa: F401
