"""MI355X-native multi-product-expansion imaginary-time eigensolver.

Hot path in hand-written HIP for gfx950 behind the C ABI of ``include/mpe.h``
(``libmpe.so`` in this directory); this package holds the ctypes binding, a
``Plan`` over torch device tensors and the step-size driver.
"""
from ._lib import MpeError, coefficients, lib  # noqa: F401
from .solver import Batch, Plan, SolveResult, solve, solve_ladder  # noqa: F401

__all__ = ["Plan", "Batch", "solve", "solve_ladder", "SolveResult", "coefficients", "MpeError", "lib"]
