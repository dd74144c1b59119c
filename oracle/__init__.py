"""CPU oracle for the nonlinear ship-wave residual and its Newton-Krylov solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow FP64 implementation
written from the paper's equations.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product library never
does, and shares no code with it.
"""
from .problem import Problem, flat_state, rule_weights, weights  # noqa: F401
from .equations import residual, residual_parts, row_scale  # noqa: F401
