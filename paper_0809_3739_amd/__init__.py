"""MI355X-native multi-product-expansion imaginary-time eigensolver.

Hot path in hand-written HIP for gfx950 behind the C ABI of ``include/mpe.h``
(``libmpe.so`` in this directory); this package holds the ctypes binding, a
``Plan`` over torch device tensors and the step-size driver.

Typical use (lowest 120 states of a potential V, float64 array [nz][ny][nx])::

    import paper_0809_3739_amd as P
    p32 = P.Plan(grid, box, 120, 12, "fp32", n_guard=8)    # order-12 expansion
    p64 = P.Plan(grid, box, 120, 12, "fp64", n_guard=8)
    for p in (p32, p64):
        p.set_potential(V)
    p32.set_gemm_precision("fp32")
    psi = p32.new_states(start)                             # [128][nz][ny][nx] on the GPU
    r = P.solve_ladder(p32, p64, psi, gamma=1e-8, lock32=3e-8, lock64=1e-9)
    r.eig[:120], r.rh[:120], r.psi                          # Ritz values, R^H, float64 states

``Plan.iterate`` is one fused step + orthonormalisation + Rayleigh-Ritz +
variances (replayed from a hipGraph); ``solve`` runs the step-size protocol in
one precision; ``Batch`` advances many uneven systems together;
``warmstart.WarmStartNet`` is the learned start.
"""
from ._lib import MpeError, coefficients, lib  # noqa: F401
from .solver import Batch, Plan, SolveResult, solve, solve_ladder  # noqa: F401

__all__ = ["Plan", "Batch", "solve", "solve_ladder", "SolveResult", "coefficients", "MpeError", "lib"]
