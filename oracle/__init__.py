"""Plain FP64 CPU oracle for the CPR Euler hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything under this directory; only the test suite, the smoke check
and the benchmark's CPU-baseline leg use it. It shares no code with the HIP
library: its tables, fluxes, residual, time stepping, limiter and adjoint are
written here from the paper's definitions, in NumPy float64, with no blocking,
fusion or reordering beyond what those definitions state.

Paper: Zimmerman, Regele, Wie, "A Comparative Study of 2D Numerical Methods
with GPU Computing" (arXiv:1709.01619).

Modules
  tables   Gauss-Legendre points, Lagrange derivative/extrapolation rows,
           Radau correction-function derivatives (Section 2.2).
  euler    Euler fluxes, ideal-gas pressure, flux Jacobians, characteristic
           eigenvectors, Rusanov flux (Section 2, Section 4).
  cpr      Grid, CPR residual (Section 2.2, differential form), SSP-RK3,
           CFL time step (Section 4), integrals and error norms.
  limiter  TVB minmod limiter on characteristic variables (Section 2.6).
  adjoint  Hand-written discrete adjoint of the residual and of one RK step.
  deviation The same residual written as deviations from a per-line
           reference state (the form the float32 residual evaluates).

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, invariants, library routines or a 50-digit brute force,
except where its docstring says "parity unpinned".
"""

from . import tables, euler, cpr, limiter, adjoint, deviation  # noqa: F401
