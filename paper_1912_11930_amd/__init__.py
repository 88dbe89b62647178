"""MI355X-native block Conjugate Gradients over *-subalgebras.

Dreier & Engwer, "Strategies for the vectorized Block Conjugate Gradients
method": Algorithm 1 (stabilised block CG, Section 3) for the classical
(block), global, parallel and hybrid *-subalgebras of Section 2, as HIP
kernels for gfx950 behind the C ABI of include/bcg.h.
"""
from ._capi import BCGError, LIB_PATH  # noqa: F401
from .autograd import BCGSolve, StencilValues  # noqa: F401
from .solver import (BCG, solve_noalloc, stencil, stencil_brick_schedule, stencil_kappa_vjp,  # noqa: F401
                     stencil_nnz, stencil_schedule)
