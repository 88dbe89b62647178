"""FP64 CPU oracle for block Conjugate Gradients over *-subalgebras.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU library is checked against. Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the GPU
library never does, and the oracle shares no code with it (the seeded input
draws in ``workload`` are the one common module, and they hold none of the
method's arithmetic).

Contents and what each follows (Dreier & Engwer, "Strategies for the
vectorized Block Conjugate Gradients method"):

* ``stencil`` -- 5-point / 7-point Dirichlet Poisson and variable-coefficient
  diffusion matrices in CSR (the paper's test problem class, Section 4; the
  coefficient recipe is this project's reading, stated in the module).
* ``bcg``     -- Algorithm 1 (stabilised block CG, Section 3) with M = I, for the
  hybrid, global, classical (block) and parallel *-subalgebras of Section 2.
* ``grad``    -- adjoint-solve gradient of a solve's output with respect to
  the matrix values and the cell coefficients.
* ``refine``  -- FP32 inner solve with FP64 outer iterative refinement
  (not in the paper; its precision policy is pinned with exact rational
  arithmetic).

Status codes match the C ABI: OK 0, NOT_CONVERGED 1, EINVAL -1, EBREAKDOWN -2.
"""

OK = 0
NOT_CONVERGED = 1
EINVAL = -1
EBREAKDOWN = -2
