"""Pins of the residual-replacement refinement oracle (CPU only).

``oracle.refine.solve_reliable`` runs one FP32 block CG iteration (the inner
policy pinned in test_oracle_refine_policy.py) and, whenever its recursive
residual has fallen by ``delta`` since the last FP64 correction, applies the
correction, replaces the residual by the FP64 true residual in a new scale
and continues with the same search direction. The scheme is not in the
paper; what fixes it:

* exact arithmetic: the replaced residual equals the recursive one, so with
  every quantity kept in FP64 (``policy32=False``) the iterates are those of
  Algorithm 1 itself (``oracle.bcg.solve``, pinned on its own against SciPy's
  CG, the Galerkin characterisation and dense solves). A wrong rescaling of
  the direction or of the line-6 product after a correction, or a restart in
  place of the continued direction, changes the iterates;
* the FP32 policy: the returned X meets the tolerance in the true FP64
  residual, recomputed here, after at least one correction;
* a right-hand side made of eigenvectors of the 2D Poisson matrix (closed
  form) is solved exactly by block CG in one iteration, and the first
  correction then ends the solve.
"""
import numpy as np
import pytest

from oracle import OK, refine
from oracle.bcg import solve as solve64
from oracle.stencil import poisson_eigenvector, stencil_csr
from workload import cell_coefficients, rhs

CASES = [("block", 0), ("global", 1), ("global", 2), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)]


def _system(k, seed=3, N=20, sigma=0.7):
    A = stencil_csr(2, N, cell_coefficients(2, N, sigma))
    return A, rhs(A.shape[0], k, "normal", seed=seed)


def _colrel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))


def reliable_fp64_mismatch(variant, p, delta=0.1, tol=1e-8, maxit=100000):
    """Largest per-column distance of the FP64-policy reliable solve from the
    plain FP64 iteration at the same iteration count; the reliable solve's
    info and the plain solve's iteration count at the same tolerance."""
    A, B = _system(8)
    Xr, ir = refine.solve_reliable(A, B, variant, p, tol=tol, delta=delta, policy32=False, maxit=maxit)
    Xo, _ = solve64(A, B, variant, p, tol=0.0, maxit=ir["iterations"])
    _, i64 = solve64(A, B, variant, p, tol=tol, maxit=10000)
    return _colrel(Xr, Xo), ir, i64["iterations"]


@pytest.mark.parametrize("variant,p", CASES)
@pytest.mark.parametrize("delta", [0.1, 0.3])
def test_fp64_policy_reproduces_the_fp64_iteration(variant, p, delta):
    """Each correction replaces the recursive residual by the true one, which
    differs from it by rounding (measured: 1e-14 of the residual early, 1e-7
    of a residual at 1e-8, i.e. at the rounding level of B); the FP64
    iteration amplifies such perturbations, and the two solutions at equal
    iteration counts differ by 3e-10 to 2.1e-9 per column at tol 1e-8, the
    stop iterations by at most 1. A wrong rescaling of the direction or of
    the line-6 product, or a restart, is off by orders of magnitude more."""
    err, ir, its64 = reliable_fp64_mismatch(variant, p, delta=delta)
    assert ir["status"] == OK and not ir["fp64_fallback"]
    assert ir["replacements"] >= 6          # one per factor delta down to 1e-8
    assert abs(ir["iterations"] - its64) <= 2
    assert err <= 1e-8, err


@pytest.mark.parametrize("variant,p", CASES)
@pytest.mark.parametrize("delta", [0.1, 1e-2])
def test_fp32_policy_meets_tolerance_in_true_residual(variant, p, delta):
    A, B = _system(8, seed=4)
    for tol in (1e-8, 1e-10):
        X, info = refine.solve_reliable(A, B, variant, p, tol=tol, delta=delta)
        assert info["status"] == OK and not info["fp64_fallback"]
        assert info["replacements"] >= 1
        R = B - A @ X
        ratio = np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0))
        assert ratio <= tol
        assert abs(ratio - info["true_ratio"]) <= 1e-12 * ratio + 1e-300
        # the FP32 iteration needs more iterations than the FP64 one, but
        # not the restarts' excess
        _, i64 = solve64(A, B, variant, p, tol=tol, maxit=10000)
        assert i64["iterations"] <= info["iterations"] <= 2 * i64["iterations"]


def test_eigenvector_block_converges_in_one_iteration():
    N, k = 12, 4
    A = stencil_csr(2, N)
    B = np.stack([poisson_eigenvector(2, N, (m, m + 1)) for m in range(1, k + 1)], axis=1)
    X, info = refine.solve_reliable(A, B, "block", 0, tol=1e-6, delta=1e-2, policy32=False)
    assert info["status"] == OK and info["iterations"] == 1 and info["replacements"] == 1
    assert np.max(np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)) <= 1e-12
