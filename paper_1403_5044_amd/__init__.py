"""MI355X-native Jacobian-free Newton-Krylov solver for nonlinear ship-wave
patterns (flow past a submerged source): HIP kernels behind a C ABI
(include/shipwave.h), with this package as a thin Python binding.

The library (libshipwave.so) is loaded on first use; nothing here computes
the method on the CPU.
"""
from .api import (Preconditioner, Problem, Server, SolveInfo, jvp, residual,  # noqa: F401
                  residual_batched, solve, zeta)
